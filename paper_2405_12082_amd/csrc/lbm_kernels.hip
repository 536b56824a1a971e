// lbm_kernels.hip -- gfx950 kernels of the D3Q27 MRT pipe stepper.
//
// Storage: populations are kept as deviations g_i = f_i - w_i in a
// section-compressed structure-of-arrays layout, state[b][i][z][k], where k
// runs over the fluid (x, y) columns of the z-invariant cross-section (no
// solid node is stored) and each (b, i, z) plane has a pitch P (multiple of
// 64 elements).  Between steps the buffer holds the post-collision values
// g*(n-1) = S^T g(n) (S: streaming with the wall), so a step is one pull
// gather, one collision and one aligned store per node: 27 loads and 27
// stores, 216 B (FP32), 108 B (FP16) or 432 B (FP64) of HBM traffic per
// fluid-node update.  The AA pattern keeps one buffer whose form alternates
// with the step parity (see StateForm); multi-step launches (graphs, the
// persistent kernel), observation of the state and the state writers live
// here too.
#include "lbm_device.h"
#include "lbm_internal.h"
#include "lbm_step.h"

namespace lbm {

// (the FP32 interpolated-wall variant asks for the bounce-back variant's 4
// waves per SIMD: without the hint it lands one register above that budget;
// the FP16 one would spill under it, or under a budget of 3 waves)
template <typename T, int BLOCK, bool WALL>
__global__ __launch_bounds__(BLOCK) LBM_OCCUPANCY __attribute__((amdgpu_waves_per_eu(WALL && sizeof(T) == 4 ? 4 : 1)))
void k_step(const Geom g, const Tiles t, const T *__restrict__ src, T *__restrict__ dst, int step_off)
{
    __shared__ float lref[href_lds_floats<T, BLOCK>()];
    const TileCoord tc = decode_tile(t, BLOCK);
    if (tc.k >= g.ncol) return;
    step_tile<T, STEP_AB, WALL>(g, t, tc, src, dst, *g.step_dev + step_off, lref + 27 * threadIdx.x);
}

// AA pattern: one buffer, updated in place (no __restrict__: reads and
// writes share it)
template <typename T, int BLOCK, int MODE>
__global__ __launch_bounds__(BLOCK) LBM_OCCUPANCY void k_step_aa(const Geom g, const Tiles t, T *buf, int step_off)
{
    __shared__ float lref[href_lds_floats<T, BLOCK>()];
    const TileCoord tc = decode_tile(t, BLOCK);
    if (tc.k >= g.ncol) return;
    step_tile<T, MODE>(g, t, tc, buf, buf, *g.step_dev + step_off, lref + 27 * threadIdx.x);
}

// Barrier of one group of workgroups inside a cooperative launch (all
// workgroups are co-resident).  Each group owns whole pipes, and a pipe's
// step n+1 reads only that pipe's step n, so the groups never wait for each
// other.  gb[0]: arrivals, gb[1]: generation, gb[2..3]: the tile counters
// of even and odd steps (one 128-byte line per group, so the atomics of
// different groups go to different lines); err[0]: error flag shared by all
// groups.  After the workgroup barrier one thread fences at agent scope
// (the release writes this XCD's L2 back, covering the stores of every wave
// of the workgroup) and arrives; the last arrival clears the tile counter
// of the step just finished (next used two steps later) before it bumps the
// generation.  The wait is bounded: on timeout the error flag is set and
// every workgroup that sees it leaves the step loop, so the grid always
// drains.
__device__ __forceinline__ bool group_barrier(unsigned *gb, unsigned *err, unsigned members, unsigned *done_counter)
{
    __syncthreads();
    __shared__ int ok;
    if (threadIdx.x == 0) {
        __threadfence();
        ok = __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u;
        if (ok) {
            const unsigned gen = __hip_atomic_load(&gb[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned arrived = __hip_atomic_fetch_add(&gb[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            if (arrived == members - 1) {
                __hip_atomic_store(&gb[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(done_counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_add(&gb[1], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                unsigned spins = 0;
                while (__hip_atomic_load(&gb[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                    __builtin_amdgcn_s_sleep(8);
                    if (++spins > (1u << 21)) {
                        __hip_atomic_fetch_or(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        ok = 0;
                        break;
                    }
                }
            }
        }
        __threadfence();
    }
    __syncthreads();
    return ok != 0;
}

// n time steps in one launch.  Workgroup w belongs to group w / per_group;
// group q owns pipes [q * pipes_per_group, ...).  Within a step the group's
// workgroups take tickets of PERSIST_CHUNK consecutive tiles from the
// group's counter (dynamic balance: a slower CU takes fewer tiles; the next
// ticket is requested before the current tiles run, hiding the atomic's
// latency), then meet at the group barrier before the next step.  Buffers
// alternate: step j reads buf[(par + j) & 1].  AA pattern: one buffer
// (buf0), par is the parity of the first step.
constexpr int PERSIST_CHUNK = 2;
template <typename T, int BLOCK, bool AA, bool WALL>
__global__ __launch_bounds__(BLOCK) void k_step_persistent(const Geom g, const Tiles t, T *buf0, T *buf1, int par,
                                                           int nsteps, unsigned *bar, int per_group,
                                                           int pipes_per_group)
{
    const int q = blockIdx.x / per_group;
    const int per_pipe = (int)t.count();
    const int b_lo = q * pipes_per_group;
    const int b_hi = min(t.nb, b_lo + pipes_per_group);
    const int first = b_lo * per_pipe, ntiles = (b_hi - b_lo) * per_pipe;
    unsigned *gb = bar + 32 * (1 + q);
    const long long n0 = *g.step_dev;
    __shared__ int ticket;
    __shared__ float lref[href_lds_floats<T, BLOCK>()];
    float *mine = lref + 27 * threadIdx.x;
    for (int j = 0; j < nsteps; ++j) {
        const T *src = ((par + j) & 1) ? buf1 : buf0;
        T *dst = ((par + j) & 1) ? buf0 : buf1;
        unsigned *ctr = &gb[2 + (j & 1)];
        if (threadIdx.x == 0) ticket = (int)__hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        int cur = ticket;
        while (cur * PERSIST_CHUNK < ntiles) {
            __syncthreads();  // every thread has read the ticket before it is replaced
            int nxt = 0;
            if (threadIdx.x == 0) nxt = (int)__hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const int lo = cur * PERSIST_CHUNK, hi = min(lo + PERSIST_CHUNK, ntiles);
            for (int tile = lo; tile < hi; ++tile) {
                const TileCoord tc = tile_coord(t, first + tile, BLOCK);
                if (tc.k >= g.ncol) continue;
                if constexpr (AA) {
                    if ((par + j) & 1)
                        step_tile<T, STEP_AA_ODD>(g, t, tc, buf0, buf0, n0 + j, mine);
                    else
                        step_tile<T, STEP_AA_EVEN>(g, t, tc, buf0, buf0, n0 + j, mine);
                } else {
                    step_tile<T, STEP_AB, WALL>(g, t, tc, src, dst, n0 + j, mine);
                }
            }
            if (threadIdx.x == 0) ticket = nxt;
            __syncthreads();
            cur = ticket;
        }
        if (j + 1 < nsteps && !group_barrier(gb, bar, (unsigned)per_group, ctr)) break;
    }
}

// Practical bandwidth ceiling of the step's access pattern: the same tiles,
// 27 aligned loads and 27 non-temporal stores per fluid node, no arithmetic.
template <typename T, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_stream_copy(const Geom g, const Tiles t, const T *__restrict__ src,
                                                        T *__restrict__ dst)
{
    const TileCoord tc = decode_tile(t, BLOCK);
    const int k = tc.k;
    if (k >= g.ncol) return;
    const char *pin = reinterpret_cast<const char *>(src + (size_t)tc.b * g.pipe);
    char *pout = reinterpret_cast<char *>(dst + (size_t)tc.b * g.pipe);
    const size_t pbytes = (size_t)g.pstride * sizeof(T);
    const unsigned rowb = (unsigned)g.P * sizeof(T);
    const int z0 = tc.zc * t.zchunk;
    const int z1 = min(z0 + t.zchunk, g.nz);
    for (int z = z0; z < z1; ++z) {
        const unsigned off = (unsigned)z * rowb + (unsigned)k * sizeof(T);
        T v[27];
#pragma unroll
        for (int i = 0; i < 27; ++i) v[i] = *reinterpret_cast<const T *>(pin + i * pbytes + off);
#pragma unroll
        for (int i = 0; i < 27; ++i) __builtin_nontemporal_store(v[i], reinterpret_cast<T *>(pout + i * pbytes + off));
    }
}

// ---------------------------------------------------------------- observe
// Gather of the current state g(n) and its moments: dense outputs and FP64
// partial sums for the diagnostics, the velocity statistics and the energy.
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <int BLOCK, int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *lds /* [BLOCK/64][NV] */)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = wave_sum(v[q]);
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < NV; ++q) lds[wid * NV + q] = v[q];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int w = 1; w < BLOCK / 64; ++w)
#pragma unroll
            for (int q = 0; q < NV; ++q) v[q] += lds[w * NV + q];
}

template <typename T, int BLOCK, int FORM, bool WALL>
__global__ __launch_bounds__(BLOCK) void k_observe(const Geom g, const Tiles t, const T *__restrict__ state,
                                                    const ObserveArgs o, int step_off)
{
    const TileCoord tc = decode_tile(t, BLOCK);
    const int k = tc.k;
    const bool active = k < g.ncol;
    const long long n = *g.step_dev + step_off;
    using R = typename RealOf<T>::type;
    const R sig = sigma_of<R>(g, n);
    double dsum[5] = {0, 0, 0, 0, 0};
    double esum[1] = {0};
    double psum[4] = {0, 0, 0, 0};
    int cnt = 0;
    __shared__ float lref[href_lds_floats<T, BLOCK>()];
    if (active) {
        Pull<T, WALL> p = make_pull<T, WALL>(state + (size_t)tc.b * g.pipe, (size_t)g.pstride, g.nbr, g.P, k,
                                             g.bcoef, g.href, lref + 27 * threadIdx.x, g.check);
        const Shape<R> sh = shape_of<R>(g, tc.b, k);
        const unsigned xy = g.colxy[k];
        int x = xy & 0xffff, y = xy >> 16;
        if (!check_ok(g.check, x < g.nx && y < g.ny, CHK_INDEX)) x = y = 0;
        const size_t plane = (size_t)g.nx * g.ny;
        const unsigned rowb = (unsigned)g.P * sizeof(T);
        const int z0 = tc.zc * t.zchunk;
        const int z1 = min(z0 + t.zchunk, g.nz);
        for (int z = z0; z < z1; ++z) {
            R v[27];
            pull_opaque<true>(p);
            gather<T, FORM, WALL>(p, (unsigned)z * rowb, (unsigned)wrap_m(z, g.nz) * rowb, (unsigned)wrap_p(z, g.nz) * rowb, v);
            R ax, ay, az;
            body_force<R>(g, z, sig, sh.px, sh.py, sh.pq, ax, ay, az);
            const Moments<R> m = moments_of<R>(v);
            const R rho = R(1) + m.dr;
            const R inv = rcp_r(rho);
            const R ux = m.jx * inv + R(0.5) * ax, uy = m.jy * inv + R(0.5) * ay, uz = m.jz * inv + R(0.5) * az;
            const size_t node = ((size_t)tc.b * g.nz + z) * plane + (size_t)y * g.nx + x;
            if (o.flags & OBS_MOMENTS) {
                if (o.rho) o.rho[node] = rho;
                if (o.u) {
                    const size_t ub = ((size_t)tc.b * 3 * g.nz + z) * plane + (size_t)y * g.nx + x;
                    const size_t us = (size_t)g.nz * plane;
                    o.u[ub] = ux;
                    o.u[ub + us] = uy;
                    o.u[ub + 2 * us] = uz;
                }
            }
            if (o.flags & OBS_POPS) {
                const size_t pb = ((size_t)tc.b * 27 * g.nz + z) * plane + (size_t)y * g.nx + x;
                const size_t ps = (size_t)g.nz * plane;
#pragma unroll
                for (int i = 0; i < 27; ++i) o.pops[pb + i * ps] = v[i];
            }
            if (o.flags & OBS_DIAG) {
                dsum[0] += (double)m.dr;
                dsum[1] += (double)m.jx;
                dsum[2] += (double)m.jy;
                dsum[3] += (double)m.jz;
                int bad = 0;
#pragma unroll
                for (int i = 0; i < 27; ++i) bad += !isfinite(v[i]);
                dsum[4] += (double)bad;
            }
            if (o.flags & OBS_PROFILE) {
                const double w = (double)uz;
                psum[0] += w;
                psum[1] += w * w;
                psum[2] += w * w * w;
                psum[3] += w * w * w * w;
            }
            if (o.flags & OBS_ENERGY) esum[0] += 0.5 * (double)rho * (double)uz * (double)uz;
            ++cnt;
        }
        if (o.flags & OBS_PROFILE) {
            double *pp = o.prof_part + (((size_t)tc.b * t.nzc + tc.zc) * g.P + k) * 5;
            pp[0] = psum[0];
            pp[1] = psum[1];
            pp[2] = psum[2];
            pp[3] = psum[3];
            pp[4] = (double)cnt;
        }
    }
    const size_t tile = ((size_t)tc.b * t.nzc + tc.zc) * t.nkb + tc.kb;
    if (o.flags & OBS_DIAG) {
        __shared__ double lds[(BLOCK / 64) * 5];
        // fluid-node count enters sum rho = N + sum dr
        dsum[0] += (double)cnt;
        block_sum<BLOCK, 5>(dsum, lds);
        if (threadIdx.x == 0)
            for (int q = 0; q < 5; ++q) o.diag_part[tile * 5 + q] = dsum[q];
        __syncthreads();
    }
    if (o.flags & OBS_ENERGY) {
        __shared__ double lde[BLOCK / 64];
        block_sum<BLOCK, 1>(esum, lde);
        if (threadIdx.x == 0) o.energy_part[tile] = esum[0];
    }
}

// fixed-order reduction of per-tile partials: one block per pipe
template <int NV>
__global__ __launch_bounds__(256) void k_reduce_tiles(const double *__restrict__ part, long long tiles_per_pipe,
                                                      double *__restrict__ out)
{
    __shared__ double lds[256 * NV];
    const int b = blockIdx.x;
    double acc[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) acc[q] = 0.0;
    for (long long t = threadIdx.x; t < tiles_per_pipe; t += 256)
#pragma unroll
        for (int q = 0; q < NV; ++q) acc[q] += part[((size_t)b * tiles_per_pipe + t) * NV + q];
#pragma unroll
    for (int q = 0; q < NV; ++q) lds[threadIdx.x * NV + q] = acc[q];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s)
#pragma unroll
            for (int q = 0; q < NV; ++q) lds[threadIdx.x * NV + q] += lds[(threadIdx.x + s) * NV + q];
        __syncthreads();
    }
    if (threadIdx.x == 0)
#pragma unroll
        for (int q = 0; q < NV; ++q) out[b * NV + q] = lds[q];
}

// acc[b] += scale * (sum of the pipe's tile partials), fixed order
__global__ __launch_bounds__(256) void k_accumulate_tiles(const double *__restrict__ part, long long tiles_per_pipe,
                                                          double scale, double *__restrict__ acc)
{
    __shared__ double lds[256];
    const int b = blockIdx.x;
    double s = 0.0;
    for (long long t = threadIdx.x; t < tiles_per_pipe; t += 256) s += part[(size_t)b * tiles_per_pipe + t];
    lds[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) lds[threadIdx.x] += lds[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) acc[b] += scale * lds[0];
}

// acc[b][k][5] += sum over z-chunks of the per-chunk partials, in order
__global__ __launch_bounds__(256) void k_reduce_profile(const double *__restrict__ part, double *__restrict__ acc,
                                                        int nzc, int P, int ncol, int B)
{
    const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (long long)B * ncol) return;
    const int b = (int)(idx / ncol), k = (int)(idx % ncol);
    double s[5] = {0, 0, 0, 0, 0};
    for (int zc = 0; zc < nzc; ++zc) {
        const double *p = part + (((size_t)b * nzc + zc) * P + k) * 5;
#pragma unroll
        for (int q = 0; q < 5; ++q) s[q] += p[q];
    }
    double *a = acc + ((size_t)b * P + k) * 5;
#pragma unroll
    for (int q = 0; q < 5; ++q) a[q] += s[q];
}

// ---------------------------------------------------------------- state writers
// Writers of a state g in a buffer form: FORM_N stores g_j(y) in slot j;
// FORM_S stores in slot j of node y the value that the pull reads: g_j(y +
// c_j) when y + c_j is fluid; else (a wall link of node y, population i =
// opp(j)) the value F with pull(F) = g_i(y): F = g_i(y) for the bounce-back,
// and for the interpolated wall F solves c F + (1 - c) X = g_i(y), where X is
// g_i(y + c_i) (own-node mode, y + c_i fluid: slot i of y is pulled by y + c_i)
// or g_j(y) (far mode: slot j of y + c_i is pulled back by y); when y + c_i is
// solid too, F and slot i of y are the two wall values of y along this line
// and solve a 2x2 system.  FORM_W: FORM_S with slots j and opp(j) exchanged.
// Computed in FP64, stored in the buffer's type.
__device__ __forceinline__ int wrap_z(int z, int dz, int nz) { return dz == 0 ? z : (dz > 0 ? wrap_p(z, nz) : wrap_m(z, nz)); }

struct SrcDense {  // populations [27][nz][ny][nx] of one pipe (float)
    const float *pops;
    size_t plane, popstride;
    const unsigned *colxy;
    int nx;
    template <int D> __device__ double get(int col, int z) const
    {
        const unsigned xy = colxy[col];
        return (double)pops[D * popstride + (size_t)z * plane + (size_t)(xy >> 16) * nx + (xy & 0xffff)];
    }
};

struct SrcEq {  // f^eq(1, (0, 0, u0(column))) - w, in FP64 (eq2: the second-order equilibrium)
    const double *u0;
    int eq2;
    template <int D> __device__ double get(int col, int) const
    {
        if (eq2) return feq2_dev_z<D, double>(u0[col]);
        const Axis<double> zero = axis_factors(0.0);
        return feq_dev<D, double>(0.0, zero, zero, axis_factors(u0[col]));
    }
};

template <typename T, int FORM, typename Src, int J = 0>
__device__ __forceinline__ void write_slots(T *pipe, const Geom &g, const int (&col)[9], const Src &src, int k, int z)
{
    double v;
    if constexpr (FORM == FORM_N) {
        v = src.template get<J>(k, z);
    } else {
        constexpr int j = FORM == FORM_W ? OPP(J) : J;  // S-form slot stored in physical slot J
        constexpr int d = NSLOT(CX(j), CY(j));
        const int sc = col[d];
        if (sc >= 0) {
            v = src.template get<j>(sc, wrap_z(z, CZ(j), g.nz));
        } else {
            constexpr int i = OPP(j);
            v = src.template get<i>(k, z);  // bounce-back
            if constexpr (d != 4) {
                if (g.bcoef) {
                    const double cf = g.bcoef[d * g.P + k];
                    if (cf != 1.0) {
                        const double gj = src.template get<j>(k, z);
                        if (cf < 0.0) {
                            const double c = -cf;
                            v = (v - (1.0 - c) * gj) / c;
                        } else {
                            const int sf = col[8 - d];
                            if (sf >= 0) {
                                v = (v - (1.0 - cf) * src.template get<i>(sf, wrap_z(z, CZ(i), g.nz))) / cf;
                            } else {
                                const double c2 = g.bcoef[(8 - d) * g.P + k];
                                v = (c2 * v - (1.0 - cf) * gj) / (cf * c2 - (1.0 - cf) * (1.0 - c2));
                            }
                        }
                    }
                }
            }
        }
    }
    using R = typename RealOf<T>::type;
    // FP16: the reference of the value's producer (see the codecs): FORM_S /
    // FORM_W hold values of this node (population J, FORM_W: opp(J)); FORM_N
    // holds g_J(y), produced by y - c_J as g*_J, or by y as g*_opp(J) where
    // y - c_J is solid
    R ref = R(0);
    if constexpr (sizeof(T) == 2) {
        if constexpr (FORM == FORM_N) {
            const int pc = col[NSLOT(-CX(J), -CY(J))];
            ref = pc >= 0 ? g.href[CZI(CZ(J)) * g.P + pc] : g.href[CZI(-CZ(J)) * g.P + k];
        } else {
            ref = g.href[CZI(FORM == FORM_W ? -CZ(J) : CZ(J)) * g.P + k];
        }
    }
    Codec<T>::template st<J>(reinterpret_cast<char *>(pipe + (size_t)J * g.pstride), (unsigned)(z * g.P + k) * sizeof(T),
                             (R)v, ref);
    if constexpr (J + 1 < 27) write_slots<T, FORM, Src, J + 1>(pipe, g, col, src, k, z);
}

// initial state f = f^eq(1, (0, 0, u0(r))) (u0 = 0: rest)
template <typename T, int FORM>
__global__ __launch_bounds__(256) void k_init(const Geom g, const double *__restrict__ u0, T *__restrict__ state)
{
    const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
    const long long total = (long long)g.B * g.nz * g.ncol;
    if (idx >= total) return;
    const int k = (int)(idx % g.ncol);
    const long long r = idx / g.ncol;
    const int z = (int)(r % g.nz), b = (int)(r / g.nz);
    int col[9];
    load_columns(g, k, col);
    write_slots<T, FORM>(state + (size_t)b * g.pipe, g, col, SrcEq{u0, kind_eq2(g.kind) ? 1 : 0}, k, z);
}

template <typename T, int FORM>
__global__ __launch_bounds__(256) void k_set_pops(const Geom g, const float *__restrict__ pops, T *__restrict__ state)
{
    const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
    const long long total = (long long)g.B * g.nz * g.ncol;
    if (idx >= total) return;
    const int k = (int)(idx % g.ncol);
    const long long r = idx / g.ncol;
    const int z = (int)(r % g.nz), b = (int)(r / g.nz);
    int col[9];
    load_columns(g, k, col);
    const size_t plane = (size_t)g.nx * g.ny, popstride = (size_t)g.nz * plane;
    const SrcDense src{pops + (size_t)b * 27 * popstride, plane, popstride, g.colxy, g.nx};
    write_slots<T, FORM>(state + (size_t)b * g.pipe, g, col, src, k, z);
}

__global__ void k_fill(uint32_t *p, size_t n)
{
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = 0u;
}
__global__ void k_copy(uint4 *dst, const uint4 *src, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) dst[i] = src[i];
}
__global__ void k_set_step(long long *p, long long v, int add)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = add ? *p + v : v;
}

// ---------------------------------------------------------------- launchers
static int grid_of(const Tiles &t) { return (int)(t.count() * t.nb); }

template <typename T, bool WALL>
static hipError_t step_wall(const Geom &g, const Tiles &t, const void *src, void *dst, int off, hipStream_t s)
{
    const dim3 grid(grid_of(t));
    switch (t.block) {
    case 64: hipLaunchKernelGGL((k_step<T, 64, WALL>), grid, dim3(64), 0, s, g, t, (const T *)src, (T *)dst, off); break;
    case 128:
        hipLaunchKernelGGL((k_step<T, 128, WALL>), grid, dim3(128), 0, s, g, t, (const T *)src, (T *)dst, off);
        break;
    case 512:
        hipLaunchKernelGGL((k_step<T, 512, WALL>), grid, dim3(512), 0, s, g, t, (const T *)src, (T *)dst, off);
        break;
    default:
        hipLaunchKernelGGL((k_step<T, 256, WALL>), grid, dim3(256), 0, s, g, t, (const T *)src, (T *)dst, off);
        break;
    }
    return hipGetLastError();
}
template <typename T>
static hipError_t step_t(const Geom &g, const Tiles &t, const void *src, void *dst, int off, hipStream_t s)
{
    return g.bcoef ? step_wall<T, true>(g, t, src, dst, off, s) : step_wall<T, false>(g, t, src, dst, off, s);
}

// the copy runs in the step's tiles: its block size must be the step's
template <typename T>
static hipError_t copy_t(const Geom &g, const Tiles &t, const void *src, void *dst, hipStream_t s)
{
    const dim3 grid(grid_of(t));
    const T *a = (const T *)src;
    T *b = (T *)dst;
    switch (t.block) {
    case 64: hipLaunchKernelGGL((k_stream_copy<T, 64>), grid, dim3(64), 0, s, g, t, a, b); break;
    case 128: hipLaunchKernelGGL((k_stream_copy<T, 128>), grid, dim3(128), 0, s, g, t, a, b); break;
    case 512: hipLaunchKernelGGL((k_stream_copy<T, 512>), grid, dim3(512), 0, s, g, t, a, b); break;
    default: hipLaunchKernelGGL((k_stream_copy<T, 256>), grid, dim3(256), 0, s, g, t, a, b); break;
    }
    return hipGetLastError();
}

hipError_t launch_stream_copy(int storage, const Geom &g, const Tiles &t, const void *src, void *dst, hipStream_t s)
{
    if (storage == 2) return copy_t<double>(g, t, src, dst, s);
    return storage == 1 ? copy_t<unsigned short>(g, t, src, dst, s) : copy_t<float>(g, t, src, dst, s);
}

template <typename T, int BLOCK, int MODE>
static void step_aa_t(const Geom &g, const Tiles &t, void *buf, int off, hipStream_t s)
{
    hipLaunchKernelGGL((k_step_aa<T, BLOCK, MODE>), dim3(grid_of(t)), dim3(BLOCK), 0, s, g, t, (T *)buf, off);
}
template <typename T, int MODE>
static hipError_t step_aa_block(const Geom &g, const Tiles &t, void *buf, int off, hipStream_t s)
{
    switch (t.block) {
    case 64: step_aa_t<T, 64, MODE>(g, t, buf, off, s); break;
    case 128: step_aa_t<T, 128, MODE>(g, t, buf, off, s); break;
    case 512: step_aa_t<T, 512, MODE>(g, t, buf, off, s); break;
    default: step_aa_t<T, 256, MODE>(g, t, buf, off, s); break;
    }
    return hipGetLastError();
}
template <typename T>
static hipError_t step_aa_mode(const Geom &g, const Tiles &t, void *buf, int odd, int off, hipStream_t s)
{
    return odd ? step_aa_block<T, STEP_AA_ODD>(g, t, buf, off, s) : step_aa_block<T, STEP_AA_EVEN>(g, t, buf, off, s);
}
hipError_t launch_step_aa(int storage, const Geom &g, const Tiles &t, void *buf, int odd, int off, hipStream_t s)
{
    if (storage == 2) return step_aa_mode<double>(g, t, buf, odd, off, s);
    return storage == 1 ? step_aa_mode<__half>(g, t, buf, odd, off, s) : step_aa_mode<float>(g, t, buf, odd, off, s);
}

template <typename T, int BLOCK, bool AA, bool WALL>
static hipError_t persistent_t(const Geom &g, const Tiles &t, void *b0, void *b1, int par, int nsteps, unsigned *bar,
                               int blocks, int per_group, int ppg, int coop, hipStream_t s)
{
    Geom gg = g;
    Tiles tt = t;
    T *p0 = (T *)b0, *p1 = (T *)b1;
    void *args[] = {&gg, &tt, &p0, &p1, &par, &nsteps, &bar, &per_group, &ppg};
    void (*fn)(const Geom, const Tiles, T *, T *, int, int, unsigned *, int, int) =
        &k_step_persistent<T, BLOCK, AA, WALL>;
    if (coop) return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(fn), dim3(blocks), dim3(BLOCK), args, 0, s);
    return hipLaunchKernel(reinterpret_cast<const void *>(fn), dim3(blocks), dim3(BLOCK), args, 0, s);
}

template <typename T, bool AA, bool WALL>
static hipError_t persistent_block(const Geom &g, const Tiles &t, void *b0, void *b1, int par, int nsteps, unsigned *bar,
                                   int blocks, int per_group, int ppg, int coop, hipStream_t s)
{
    switch (t.block) {
    case 64: return persistent_t<T, 64, AA, WALL>(g, t, b0, b1, par, nsteps, bar, blocks, per_group, ppg, coop, s);
    case 128: return persistent_t<T, 128, AA, WALL>(g, t, b0, b1, par, nsteps, bar, blocks, per_group, ppg, coop, s);
    case 512: return persistent_t<T, 512, AA, WALL>(g, t, b0, b1, par, nsteps, bar, blocks, per_group, ppg, coop, s);
    default: return persistent_t<T, 256, AA, WALL>(g, t, b0, b1, par, nsteps, bar, blocks, per_group, ppg, coop, s);
    }
}
// kinds: two buffers + bounce-back, AA + bounce-back, two buffers + interpolated wall
template <typename T>
static hipError_t persistent_pattern(int aa, const Geom &g, const Tiles &t, void *b0, void *b1, int par, int nsteps,
                                     unsigned *bar, int blocks, int per_group, int ppg, int coop, hipStream_t s)
{
    if (aa) return persistent_block<T, true, false>(g, t, b0, b1, par, nsteps, bar, blocks, per_group, ppg, coop, s);
    if (g.bcoef) return persistent_block<T, false, true>(g, t, b0, b1, par, nsteps, bar, blocks, per_group, ppg, coop, s);
    return persistent_block<T, false, false>(g, t, b0, b1, par, nsteps, bar, blocks, per_group, ppg, coop, s);
}

hipError_t launch_step_persistent(int storage, int aa, const Geom &g, const Tiles &t, void *b0, void *b1, int par,
                                  int nsteps, unsigned *bar, int blocks, int per_group, int pipes_per_group,
                                  int coop, hipStream_t s)
{
    if (storage == 2)
        return persistent_pattern<double>(aa, g, t, b0, b1, par, nsteps, bar, blocks, per_group, pipes_per_group, coop, s);
    if (storage == 1)
        return persistent_pattern<__half>(aa, g, t, b0, b1, par, nsteps, bar, blocks, per_group, pipes_per_group, coop, s);
    return persistent_pattern<float>(aa, g, t, b0, b1, par, nsteps, bar, blocks, per_group, pipes_per_group, coop, s);
}

template <typename T, int BLOCK, bool AA, bool WALL> static int occ_t()
{
    int n = 0;
    void (*fn)(const Geom, const Tiles, T *, T *, int, int, unsigned *, int, int) =
        &k_step_persistent<T, BLOCK, AA, WALL>;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void *>(fn), BLOCK, 0) != hipSuccess)
        return 0;
    return n;
}
template <typename T, bool AA, bool WALL> static int occ_block(int block)
{
    return block == 64    ? occ_t<T, 64, AA, WALL>()
           : block == 128 ? occ_t<T, 128, AA, WALL>()
           : block == 512 ? occ_t<T, 512, AA, WALL>()
                          : occ_t<T, 256, AA, WALL>();
}
template <typename T> static int occ_pattern(int aa, int wall, int block)
{
    if (aa) return occ_block<T, true, false>(block);
    return wall ? occ_block<T, false, true>(block) : occ_block<T, false, false>(block);
}
int persistent_blocks_per_cu(int storage, int aa, int wall, int block)
{
    return storage == 2 ? occ_pattern<double>(aa, wall, block)
                        : (storage == 1 ? occ_pattern<__half>(aa, wall, block) : occ_pattern<float>(aa, wall, block));
}

hipError_t launch_step(int storage, const Geom &g, const Tiles &t, const void *src, void *dst, int off, hipStream_t s)
{
    if (g.kind != KIND_MRT6) return launch_step_kind(storage, g, t, src, dst, off, s);
    if (storage == 2) return step_t<double>(g, t, src, dst, off, s);
    return storage == 1 ? step_t<__half>(g, t, src, dst, off, s) : step_t<float>(g, t, src, dst, off, s);
}

template <typename T, int FORM, bool WALL = false>
static void observe_t(const Geom &g, const Tiles &t, const void *state, const ObserveArgs &o, int off, hipStream_t s)
{
    hipLaunchKernelGGL((k_observe<T, 256, FORM, WALL>), dim3(grid_of(t)), dim3(256), 0, s, g, t, (const T *)state, o,
                       off);
}
template <typename T>
static void observe_form(int form, const Geom &g, const Tiles &t, const void *state, const ObserveArgs &o, int off,
                         hipStream_t s)
{
    if (form == FORM_N)
        observe_t<T, FORM_N>(g, t, state, o, off, s);
    else if (form == FORM_W)
        observe_t<T, FORM_W>(g, t, state, o, off, s);
    else if (g.bcoef)
        observe_t<T, FORM_S, true>(g, t, state, o, off, s);
    else
        observe_t<T, FORM_S>(g, t, state, o, off, s);
}
hipError_t launch_observe(int storage, int form, const Geom &g, const Tiles &t, const void *state, const ObserveArgs &o,
                          int off, hipStream_t s)
{
    if (storage == 2)
        observe_form<double>(form, g, t, state, o, off, s);
    else if (storage == 1)
        observe_form<__half>(form, g, t, state, o, off, s);
    else
        observe_form<float>(form, g, t, state, o, off, s);
    return hipGetLastError();
}

static dim3 node_grid(const Geom &g)
{
    const long long total = (long long)g.B * g.nz * g.ncol;
    return dim3((unsigned)((total + 255) / 256));
}

template <typename T>
static void init_form(int form, const Geom &g, const double *u0, void *state, hipStream_t s)
{
    if (form == FORM_N)
        hipLaunchKernelGGL((k_init<T, FORM_N>), node_grid(g), dim3(256), 0, s, g, u0, (T *)state);
    else if (form == FORM_W)
        hipLaunchKernelGGL((k_init<T, FORM_W>), node_grid(g), dim3(256), 0, s, g, u0, (T *)state);
    else
        hipLaunchKernelGGL((k_init<T, FORM_S>), node_grid(g), dim3(256), 0, s, g, u0, (T *)state);
}
hipError_t launch_init(int storage, int form, const Geom &g, const double *u0, void *state, hipStream_t s)
{
    if (storage == 2)
        init_form<double>(form, g, u0, state, s);
    else if (storage == 1)
        init_form<__half>(form, g, u0, state, s);
    else
        init_form<float>(form, g, u0, state, s);
    return hipGetLastError();
}

template <typename T>
static void set_pops_form(int form, const Geom &g, const float *pops, void *state, hipStream_t s)
{
    if (form == FORM_N)
        hipLaunchKernelGGL((k_set_pops<T, FORM_N>), node_grid(g), dim3(256), 0, s, g, pops, (T *)state);
    else if (form == FORM_W)
        hipLaunchKernelGGL((k_set_pops<T, FORM_W>), node_grid(g), dim3(256), 0, s, g, pops, (T *)state);
    else
        hipLaunchKernelGGL((k_set_pops<T, FORM_S>), node_grid(g), dim3(256), 0, s, g, pops, (T *)state);
}
hipError_t launch_set_pops(int storage, int form, const Geom &g, const float *pops, void *state, hipStream_t s)
{
    if (storage == 2)
        set_pops_form<double>(form, g, pops, state, s);
    else if (storage == 1)
        set_pops_form<__half>(form, g, pops, state, s);
    else
        set_pops_form<float>(form, g, pops, state, s);
    return hipGetLastError();
}

hipError_t launch_reduce_diag(const Geom &g, const Tiles &t, const double *part, double *out, hipStream_t s)
{
    hipLaunchKernelGGL((k_reduce_tiles<5>), dim3(g.B), dim3(256), 0, s, part, t.count(), out);
    return hipGetLastError();
}

hipError_t launch_reduce_energy(const Geom &g, const Tiles &t, const double *part, double *out, hipStream_t s)
{
    hipLaunchKernelGGL((k_reduce_tiles<1>), dim3(g.B), dim3(256), 0, s, part, t.count(), out);
    return hipGetLastError();
}

hipError_t launch_accumulate_energy(const Geom &g, const Tiles &t, const double *part, double scale, double *acc,
                                    hipStream_t s)
{
    hipLaunchKernelGGL(k_accumulate_tiles, dim3(g.B), dim3(256), 0, s, part, t.count(), scale, acc);
    return hipGetLastError();
}

hipError_t launch_reduce_profile(const Geom &g, const Tiles &t, const double *part, double *acc, hipStream_t s)
{
    const long long n = (long long)g.B * g.ncol;
    hipLaunchKernelGGL(k_reduce_profile, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, part, acc, t.nzc, g.P,
                       g.ncol, g.B);
    return hipGetLastError();
}

hipError_t launch_fill(void *p, size_t bytes, hipStream_t s)
{
    const size_t n = bytes / 4;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (uint32_t *)p, n);
    return hipGetLastError();
}

hipError_t launch_copy(void *dst, const void *src, size_t bytes, hipStream_t s)
{
    const size_t n = bytes / 16;
    if (n == 0) return hipSuccess;
    const size_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(256), 0, s, (uint4 *)dst,
                       (const uint4 *)src, n);
    return hipGetLastError();
}

hipError_t launch_set_step(long long *p, long long v, int add, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_step, dim3(1), dim3(64), 0, s, p, v, add);
    return hipGetLastError();
}

}  // namespace lbm
