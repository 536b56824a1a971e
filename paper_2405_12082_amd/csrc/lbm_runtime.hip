// lbm_runtime.hip -- host runtime and C-ABI of the D3Q27 MRT pipe stepper.
//
// Builds the z-invariant tables of the pipe on the host (fluid-column list,
// neighbour table, trigger-force shapes of Eq. (TurbForce), log-law profile
// of the initial state, Section II.B), carves the caller's workspace and
// enqueues the kernels on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_internal.h"

using namespace lbm;

namespace {

constexpr int kMaxModes = 6;
constexpr long long kMaxSigma = 1LL << 24;   // longest forcing window (steps)
constexpr int kObsZChunk = 16;               // z planes per thread for observation kernels
#ifndef LBM_ADJ_ZCHUNK
#define LBM_ADJ_ZCHUNK 8
#endif
constexpr int kAdjZChunk = LBM_ADJ_ZCHUNK;   // z planes per thread for the adjoint step
constexpr int kMaxRing = 4096;               // ring points of the coherent-structure sampling
constexpr int kDefaultZChunk2 = 32;          // output planes per workgroup of the two-step kernel
// default threads per block by storage (turbulent pipe, graph replays: FP32
// 1.146 ms at 512 vs 1.164 ms at 256; FP16 best at 256); with the
// interpolated wall FP32 is best at 256 threads and 2 planes (1.244 ms vs
// 1.281 at 512), FP16 at 64 threads and 16 planes (paper pipe: 1.222 ms vs
// 1.422 at 256 threads: the waves with wall columns take longer, and a
// workgroup holds its slot until its slowest wave ends)
constexpr int kDefaultBlock[3] = {512, 256, 256};
constexpr int kDefaultBlockWall[3] = {256, 64, 256}, kDefaultZChunkWall[3] = {2, 16, 2};
// default z planes per thread by storage (measured on the 192^2 x 1152 pipe:
// FP32 1.173 ms at 1 plane vs 1.209 ms at 4; FP16 best at 8)
constexpr int kDefaultZChunk[3] = {1, 8, 2};

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Layout {
    std::vector<int> colx, coly;   // fluid columns, row-major (y outer, x inner)
    std::vector<int> colmap;       // [ny][nx] -> column or -1
    int ncol = 0, P = 0;
    long long pstride = 0;         // elements between the populations of one pipe
    Tiles step{}, obs{}, adj{};
    std::vector<int> box;          // two-step kernel: [tiles][FUSED_BOX] box columns
    int nt2 = 0;                   // its tiles
    size_t elem = 4;               // bytes per stored population
    size_t state_bytes = 0;
    size_t record_bytes = 0;       // one moment record of the recording step (all pipes)
    // workspace offsets
    size_t off_state[2], off_box, off_nbr, off_bcoef, off_colxy, off_fshape, off_ztab, off_sigma, off_u0, off_step, off_step2, off_bar;
    size_t off_check = 0;  // bounds-violation flags of a checked build (one word)
    size_t off_fshape64, off_ztab64, off_sigma64;  // FP64 storage only
    size_t off_href;                               // FP16 storage only
    size_t off_diag_part, off_diag_out, off_prof_part, off_prof_acc, off_energy_part, off_energy_out;
    size_t off_lam[2], off_grad_part, off_grad_col, off_grad_base, off_modes;
    size_t off_ring_nodes, off_ring_idx, off_ring_w, off_twiddle;
    size_t total = 0;
    long long n_sigma = 0;
    std::string err;
};

bool fluid_xy(const lbm_config &c, int x, int y)
{
    if (c.radius <= 0.0) return true;
    const double dx = x - 0.5 * (c.nx - 1), dy = y - 0.5 * (c.ny - 1);
    return std::sqrt(dx * dx + dy * dy) < c.radius;
}

int build_layout(const lbm_config *cfg, Layout &L)
{
    if (!cfg) {
        L.err = "config is NULL";
        return LBM_EINVAL;
    }
    const lbm_config &c = *cfg;
    char buf[256];
    auto bad = [&](const char *m) {
        L.err = m;
        return LBM_EINVAL;
    };
    if (c.nx < 1 || c.ny < 1 || c.nz < 1 || c.batch < 1) return bad("nx, ny, nz and batch must be >= 1");
    if (c.nx > 32767 || c.ny > 32767) return bad("nx and ny must be < 32768");
    if (!(c.tau > 0.5) || !std::isfinite(c.tau)) return bad("tau must be > 0.5");
    if (!std::isfinite(c.accel_z)) return bad("accel_z must be finite");
    if (c.n_modes < 0 || c.n_modes > kMaxModes) return bad("n_modes must be in 0..6");
    if (c.n_modes > 0) {
        if (!(c.period > 0.0)) return bad("period must be > 0 when n_modes > 0");
        if (c.radius <= 0.0) return bad("the trigger force needs a pipe wall (radius > 0)");
        if (!(c.l_frac > 0.0) || c.l0_frac < 0.0) return bad("l_frac must be > 0 and l0_frac >= 0");
        if (c.force_off_step > kMaxSigma) return bad("force_off_step must be <= 2^24");
    }
    if (c.storage < 0 || c.storage > 2) return bad("storage must be 0 (FP32), 1 (FP16) or 2 (FP64)");
    if (c.storage == 2 && c.adjoint == 1) return bad("the adjoint of the FP64 forward is FP64 (adjoint = 2)");
    if (c.wall != 0 && c.wall != 1) return bad("wall must be 0 (halfway bounce-back) or 1 (interpolated, Bouzidi)");
    if (c.wall == 1 && !(c.radius > 0.0)) return bad("the interpolated wall needs a pipe wall (radius > 0)");
    if (c.wall == 1 && c.pattern != 0) return bad("the interpolated wall needs the two-buffer pattern (pattern = 0)");
    if (c.pattern != 0 && c.pattern != 1) return bad("pattern must be 0 (two buffers) or 1 (AA, in place)");
    if (c.pattern == 1 && c.adjoint != 0) return bad("the adjoint needs the two-buffer pattern (pattern = 0)");
    if (c.init != 0 && c.init != 1) return bad("init must be 0 (rest) or 1 (log-law)");
    if (c.adjoint < 0 || c.adjoint > 2) return bad("adjoint must be 0 (none), 1 (FP32) or 2 (FP64)");
    if (c.init == 1 && (c.radius <= 0.0 || !(c.u_tau >= 0.0))) return bad("log-law init needs radius > 0, u_tau >= 0");
    if (c.collision != 0 && c.collision != 1) return bad("collision must be 0 (MRT) or 1 (BGK)");
    if (c.equilibrium != 0 && c.equilibrium != 1) return bad("equilibrium must be 0 (sixth order) or 1 (second order)");
    if (c.collision != 0 || c.equilibrium != 0) {
        if (c.storage == 1) return bad("the comparison schemes need FP32 or FP64 storage");
        if (c.pattern != 0) return bad("the comparison schemes need the two-buffer pattern (pattern = 0)");
        if (c.adjoint != 0) return bad("the comparison schemes have no adjoint (adjoint must be 0)");
    }
    if (c.radius > 0.0 && c.radius > 0.5 * (std::min(c.nx, c.ny) - 1))
        return bad("radius must be <= (min(nx, ny) - 1) / 2 so that the outer ring of the box is solid");
    const int sidx = (c.storage >= 0 && c.storage <= 2) ? c.storage : 0;
    const bool iwall = c.wall == 1;
    const int block = c.block ? c.block : (iwall ? kDefaultBlockWall[sidx] : kDefaultBlock[sidx]);
    if (block != 64 && block != 128 && block != 256 && block != 512) return bad("block must be 64, 128, 256 or 512");
    const int zchunk = c.zchunk ? c.zchunk : (iwall ? kDefaultZChunkWall[sidx] : kDefaultZChunk[sidx]);
    if (zchunk < 1 || zchunk > 64) return bad("zchunk must be in 1..64");

    L.colmap.assign((size_t)c.nx * c.ny, -1);
    L.colx.clear();
    L.coly.clear();
    for (int y = 0; y < c.ny; ++y)
        for (int x = 0; x < c.nx; ++x)
            if (fluid_xy(c, x, y)) {
                L.colmap[(size_t)y * c.nx + x] = (int)L.colx.size();
                L.colx.push_back(x);
                L.coly.push_back(y);
            }
    L.ncol = (int)L.colx.size();
    if (L.ncol == 0) return bad("the cross-section has no fluid column");
    // tiles of the two-step kernel: 14 x 14 interiors with a halo ring
    // (periodic wrap); tiles without an own fluid column are dropped
    L.box.clear();
    for (int ty = 0; ty * FUSED_IN < c.ny; ++ty)
        for (int tx = 0; tx * FUSED_IN < c.nx; ++tx) {
            int box[FUSED_BOX];
            bool any = false;
            for (int ly = 0; ly < FUSED_BY; ++ly)
                for (int lx = 0; lx < FUSED_BX; ++lx) {
                    const int ux = tx * FUSED_IN - 1 + lx, uy = ty * FUSED_IN - 1 + ly;
                    const int x = (ux % c.nx + c.nx) % c.nx, y = (uy % c.ny + c.ny) % c.ny;
                    int v = L.colmap[(size_t)y * c.nx + x];
                    const bool interior = lx >= 1 && lx <= FUSED_IN && ly >= 1 && ly <= FUSED_IN;
                    if (v >= 0 && interior && ux < c.nx && uy < c.ny) {
                        v |= FUSED_OWNED;
                        any = true;
                    }
                    box[ly * FUSED_BX + lx] = v;
                }
            if (any) L.box.insert(L.box.end(), box, box + FUSED_BOX);
        }
    L.nt2 = (int)(L.box.size() / FUSED_BOX);
    L.P = (int)align_up((size_t)L.ncol, 64);
    // population stride: nz planes, padded by 37 x 64 elements when it is a
    // multiple of 4096 elements (then the 27 read and 27 write streams of a
    // step all start at one offset modulo 16 KiB or more; the 27-stream copy
    // of the turbulent pipe measured 1.4% slower so)
    L.pstride = (long long)c.nz * L.P;
    if (L.pstride % 4096 == 0) L.pstride += 37 * 64;
    L.elem = c.storage == 1 ? 2 : (c.storage == 2 ? 8 : 4);
    // the kernels address the state with 64-bit pipe and population bases and
    // 32-bit byte offsets within one population's region
    if (L.pstride * L.elem >= (1LL << 32)) {
        std::snprintf(buf, sizeof buf, "pipe too large: one population takes %lld bytes, must be < 4 GiB",
                      L.pstride * L.elem);
        return bad(buf);
    }
    // the adjoint state (FP32 or FP64) is addressed the same way
    const long long adj_elem = c.adjoint == 2 ? 8 : 4;
    if (c.adjoint != 0 && L.pstride * adj_elem >= (1LL << 32)) {
        std::snprintf(buf, sizeof buf, "pipe too large for the adjoint: one adjoint population takes %lld bytes, "
                      "must be < 4 GiB", L.pstride * adj_elem);
        return bad(buf);
    }
    const long long pipe_elems = 27 * L.pstride;
    L.state_bytes = align_up((size_t)pipe_elems * c.batch * L.elem, 256);
    L.record_bytes = align_up((size_t)4 * L.pstride * c.batch * (c.storage == 2 ? 8 : 4), 256);
    if (c.xcd_remap < 0 || c.xcd_remap > 4096) return bad("xcd_remap must be in 0..4096");
    L.step = Tiles{block, zchunk, (L.ncol + block - 1) / block, (c.nz + zchunk - 1) / zchunk, c.xcd_remap, 0, c.batch};
    L.obs = Tiles{256, kObsZChunk, (L.ncol + 255) / 256, (c.nz + kObsZChunk - 1) / kObsZChunk, 1, 0, c.batch};
    L.adj = Tiles{256, kAdjZChunk, (L.ncol + 255) / 256, (c.nz + kAdjZChunk - 1) / kAdjZChunk, 1, 0, c.batch};
    L.n_sigma = c.n_modes > 0 ? std::max<long long>(c.force_off_step, 0) : 0;

    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + std::max<size_t>(bytes, 1), 256);
        return o;
    };
    const size_t B = (size_t)c.batch, P = (size_t)L.P;
    L.off_state[0] = take(L.state_bytes);
    L.off_state[1] = c.pattern == 1 ? L.off_state[0] : take(L.state_bytes);  // AA: one buffer
    L.off_nbr = take(9 * P * sizeof(int));
    L.off_box = take(L.box.size() * sizeof(int));
    L.off_bcoef = c.wall == 1 ? take(9 * P * sizeof(double)) : 0;
    L.off_colxy = take(P * sizeof(unsigned));
    L.off_fshape = take(B * 3 * P * sizeof(float));
    L.off_ztab = take(2 * (size_t)c.nz * sizeof(float));
    L.off_sigma = take((size_t)L.n_sigma * sizeof(float));
    L.off_u0 = take(P * sizeof(double));
    const bool fp64 = c.storage == 2;
    L.off_fshape64 = fp64 ? take(B * 3 * P * sizeof(double)) : 0;
    L.off_ztab64 = fp64 ? take(2 * (size_t)c.nz * sizeof(double)) : 0;
    L.off_sigma64 = fp64 ? take((size_t)L.n_sigma * sizeof(double)) : 0;
    L.off_href = c.storage == 1 ? take(3 * P * sizeof(float)) : 0;
    L.off_step = take(sizeof(long long));
    L.off_step2 = take(sizeof(long long));
    L.off_check = take(sizeof(unsigned));
    L.off_bar = take(32 * sizeof(unsigned) * ((size_t)cfg->batch + 1));
    L.off_ring_nodes = take((size_t)kMaxRing * 4 * sizeof(int));
    L.off_ring_idx = take((size_t)kMaxRing * 4 * sizeof(int));
    L.off_ring_w = take((size_t)kMaxRing * 4 * sizeof(double));
    L.off_twiddle = take((size_t)kMaxRing * 2 * sizeof(double));
    const size_t obs_tiles = (size_t)L.obs.count() * B;
    L.off_diag_part = take(obs_tiles * 5 * sizeof(double));
    L.off_diag_out = take(B * 5 * sizeof(double));
    L.off_prof_part = take(B * L.obs.nzc * P * 5 * sizeof(double));
    L.off_prof_acc = take(B * P * 5 * sizeof(double));
    L.off_energy_part = take(obs_tiles * sizeof(double));
    L.off_energy_out = take(B * sizeof(double));
    if (c.adjoint) {
        const size_t lam = align_up((size_t)pipe_elems * B * (c.adjoint == 2 ? sizeof(double) : sizeof(float)), 256);
        L.off_lam[0] = take(lam);
        L.off_lam[1] = take(lam);
        L.off_grad_part = take(B * L.adj.nzc * P * 3 * sizeof(double));
        L.off_grad_col = take(B * P * 3 * sizeof(double));
        L.off_grad_base = take(B * 2 * kMaxModes * sizeof(double));
        L.off_modes = take((size_t)2 * kMaxModes * 3 * P * sizeof(double));
    } else {
        L.off_lam[0] = L.off_lam[1] = L.off_grad_part = L.off_grad_col = L.off_grad_base = L.off_modes = 0;
    }
    L.total = off;
    return LBM_OK;
}

// One mode of Eq. (TurbForce) at unit time factor and unit z-factor:
// cylindrical (F_r, F_theta, F_z) without the cos/sin(k_z 2 pi z / L)
// factors, which the kernels apply per plane.  Mode m, phase phi.
void mode_shape(const lbm_config &c, double amp, int m, double phi, int x, int y, double out[3])
{
    out[0] = out[1] = out[2] = 0.0;
    const double R = c.radius, L = (double)c.nz;
    const double l0 = c.l0_frac * R, l = c.l_frac * R;
    const double dx = x - 0.5 * (c.nx - 1), dy = y - 0.5 * (c.ny - 1);
    const double r = std::sqrt(dx * dx + dy * dy);
    if (r <= 0.0 || r < R - l0 - l || r > R - l0) return;
    const double th = std::atan2(dy, dx), a = m * (th - phi);
    const double arg = 2.0 * M_PI * (R - r - l0) / l;
    const double Fr = -amp * c.kappa * (R / r) * (c.kz * l / L) * (1.0 - std::cos(arg)) * std::cos(a);
    const double Ft = amp * (1.0 - c.kappa) * (c.kz / m) * (2.0 * M_PI * R / L) * std::sin(arg) * std::sin(a);
    const double Fz = -amp * (R / r) * std::sin(arg) * std::cos(a);
    out[0] = Fr * std::cos(th) - Ft * std::sin(th);
    out[1] = Fr * std::sin(th) + Ft * std::cos(th);
    out[2] = Fz;
}

// Interpolated wall, Eqs. (fbc1)/(fbc2): for fluid column (x, y) whose
// in-plane neighbour at offset (dx, dy) is solid, Delta in (0, 1] is the
// fraction of that link at which it crosses r = R (ray-circle
// intersection; c_z does not change r).  Coefficient of the pull (see
// pull_one): +1/(2 Delta) for Delta >= 1/2, -2 Delta for Delta < 1/2 when the
// node on the other side, (x - dx, y - dy), is fluid, else +1 (bounce-back).
double wall_coefficient(const lbm_config &c, int x, int y, int dx, int dy, bool far_fluid)
{
    const double px = x - 0.5 * (c.nx - 1), py = y - 0.5 * (c.ny - 1);
    const double a = dx * dx + dy * dy, b = 2.0 * (px * dx + py * dy), q = px * px + py * py - c.radius * c.radius;
    const double delta = (-b + std::sqrt(b * b - 4.0 * a * q)) / (2.0 * a);
    if (delta >= 0.5) return 1.0 / (2.0 * delta);
    return far_fluid ? -2.0 * delta : 1.0;
}

double loglaw(const lbm_config &c, double r)
{
    const double nu = (c.tau - 0.5) / 3.0;
    const double dp = (c.radius - r) * c.u_tau / nu;
    return c.u_tau * (dp <= 10.8 ? dp : std::log(dp) / 0.4 + 5.0);
}

}  // namespace

struct lbm_ctx {
    lbm_config cfg{};
    Layout L;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    char *ws = nullptr;
    Geom geom{};
    long long step = 0;
    int sticky = 0;
    std::string err;
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    int ppl = 1;         // pipes per step launch
    int pipe_major = 0;  // 1: each pipe group runs all steps of a call before the next group
    int graph_k[2] = {0, 0};
    hipGraphExec_t pgraph[2] = {nullptr, nullptr};  // persistent launches, per starting buffer
    int pgraph_k[2] = {0, 0};
    // two steps per launch (fuse == 2): the two-step kernel writes step n+2
    // into the other buffer, so the buffer of step n is (n + flip) & 1
    int fuse = 1;
    int flip = 0;
    Tiles2 t2{};
    // adjoint
    bool adj_ready = false;
    long long cursor = -1, obs_begin = 0, obs_end = 0;
    int lam_cur = 0;
    bool lam_nonzero = false;
    bool grad_base_set = false;  // the sweep's starting gradient has been saved
    // coherent-structure ring: host copies of the device tables (alive while
    // their asynchronous uploads run) and what they were built for
    std::vector<int> ring_nodes, ring_idx;
    std::vector<double> ring_w, twiddle;
    double ring_r0 = -1.0;
    int ring_n = 0, tw_n = 0;
    // failure watchdog of lbm_diagnostics: relative mass-drift limit (0: off)
    // and the reference masses (taken at the first diagnostics call after
    // lbm_init, lbm_load, lbm_set_populations or lbm_set_watchdog)
    double watch_tol = 0.0;
    std::vector<double> mass_ref;

    int buf(long long n) const { return (int)((n + flip) & 1); }
    void *state(long long n) const { return ws + L.off_state[buf(n)]; }
    bool can_fuse() const { return cfg.pattern == 0 && cfg.wall == 0 && cfg.storage != 2 && geom.kind == 0; }
    // form of the buffer that holds the state of step n
    int form(long long n) const { return cfg.pattern == 1 ? ((n & 1) ? FORM_W : FORM_N) : FORM_S; }
};

namespace {

int fail(lbm_ctx *c, int code, const std::string &msg)
{
    if (c) {
        c->err = msg;
        if (code == LBM_EHIP) c->sticky = 1;
    }
    return code;
}

#define HIPCHK(ctx, expr)                                                                                   \
    do {                                                                                                    \
        hipError_t e_ = (expr);                                                                             \
        if (e_ != hipSuccess)                                                                               \
            return fail(ctx, LBM_EHIP, std::string(#expr " failed: ") + hipGetErrorString(e_));             \
    } while (0)

#define CHECK_CTX(ctx)                                                                                      \
    do {                                                                                                    \
        if (!(ctx)) return LBM_EINVAL;                                                                      \
        if ((ctx)->sticky) return LBM_EHIP;                                                                 \
    } while (0)

// n steps from step index `first` for every pipe, one launch per group of
// pipes_per_launch pipes, step-major or pipe-major.  With fuse == 2, pairs
// of steps run as one two-step launch (a single step completes an odd n).
// flip: the buffer flip at `first` (flip_after gives the one after).
hipError_t launch_steps(lbm_ctx *c, long long first, int n, int flip, hipStream_t s)
{
    const int B = c->cfg.batch;
    struct Unit {
        int j, len, bi;  // first step offset, 1 or 2 steps, source buffer
    };
    std::vector<Unit> units;
    for (int j = 0; j < n;) {
        const int bi = (int)((first + j + flip) & 1);
        if (c->fuse == 2 && j + 2 <= n) {
            units.push_back({j, 2, bi});
            flip ^= 1;
            j += 2;
        } else {
            units.push_back({j, 1, bi});
            j += 1;
        }
    }
    auto one = [&](int b0, const Unit &u) {
        const int nb = std::min(c->ppl, B - b0);
        void *src = c->ws + c->L.off_state[u.bi], *dst = c->ws + c->L.off_state[u.bi ^ 1];
        if (u.len == 2) {
            Tiles2 t = c->t2;
            t.b0 = b0;
            t.nb = nb;
            return launch_step2(c->cfg.storage, c->geom, t, src, dst, u.j, s);
        }
        Tiles t = c->L.step;
        t.b0 = b0;
        t.nb = nb;
        if (c->cfg.pattern == 1)
            return launch_step_aa(c->cfg.storage, c->geom, t, src, (int)((first + u.j) & 1), u.j, s);
        return launch_step(c->cfg.storage, c->geom, t, src, dst, u.j, s);
    };
    hipError_t e = hipSuccess;
    if (c->pipe_major) {
        for (int b0 = 0; b0 < B && e == hipSuccess; b0 += c->ppl)
            for (size_t q = 0; q < units.size() && e == hipSuccess; ++q) e = one(b0, units[q]);
    } else {
        for (size_t q = 0; q < units.size() && e == hipSuccess; ++q)
            for (int b0 = 0; b0 < B && e == hipSuccess; b0 += c->ppl) e = one(b0, units[q]);
    }
    return e;
}

// the buffer flip after n more steps from the current state
int flip_after(const lbm_ctx *c, int n) { return c->flip ^ (c->fuse == 2 ? (n / 2) & 1 : 0); }

int do_step_eager(lbm_ctx *c, int n)
{
    HIPCHK(c, launch_steps(c, c->step, n, c->flip, c->stream));
    c->flip = flip_after(c, n);
    if (n > 0) HIPCHK(c, launch_set_step(const_cast<long long *>(c->geom.step_dev), n, 1, c->stream));
    c->step += n;
    return LBM_OK;
}

int observe(lbm_ctx *c, const ObserveArgs &o)
{
    HIPCHK(c, launch_observe(c->cfg.storage, c->form(c->step), c->geom, c->L.obs, c->state(c->step), o, 0, c->stream));
    return LBM_OK;
}

// workgroups of a persistent launch: groups of co-resident workgroups that
// own whole pipes, as many groups as pipes while the co-resident workgroups
// suffice, else several pipes per group
struct PersistentPlan {
    int blocks, per_group, ppg, groups;
};
int persistent_plan(lbm_ctx *c, PersistentPlan &pl)
{
    if (c->geom.kind != 0) return fail(c, LBM_EINVAL, "persistent launches run the paper's collision only");
    int dev = 0, cus = 0;
    HIPCHK(c, hipGetDevice(&dev));
    HIPCHK(c, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int aa = c->cfg.pattern == 1;
    const int per_cu = persistent_blocks_per_cu(c->cfg.storage, aa, c->cfg.wall, c->L.step.block);
    if (per_cu < 1 || cus < 1) return fail(c, LBM_EHIP, "persistent launch: occupancy query failed");
    const long long slots = (long long)per_cu * cus, per_pipe = c->L.step.count();
    const int B = c->cfg.batch;
    if (per_pipe * B > INT_MAX) return fail(c, LBM_EINVAL, "persistent launch: too many tiles for one launch");
    pl.ppg = (int)((B + slots - 1) / slots);
    pl.groups = (B + pl.ppg - 1) / pl.ppg;
    pl.per_group = (int)std::min<long long>(slots / pl.groups, per_pipe * pl.ppg);
    pl.blocks = pl.groups * pl.per_group;
    return LBM_OK;
}
// n steps from the current state as one persistent launch plus the step
// counter update (cooperative: a launch of its own; 0: a plain launch, for
// graph capture, where the grid is still sized to the co-resident
// workgroups and the barrier wait stays bounded)
hipError_t launch_persistent(lbm_ctx *c, const PersistentPlan &pl, int n, int cooperative, hipStream_t s)
{
    Tiles t = c->L.step;
    t.b0 = 0;
    t.nb = c->cfg.batch;
    const int aa = c->cfg.pattern == 1;
    unsigned *bar = (unsigned *)(c->ws + c->L.off_bar);
    hipError_t e = launch_step_persistent(c->cfg.storage, aa, c->geom, t, c->state(c->step), c->state(c->step + 1),
                                          aa ? (int)(c->step & 1) : 0, n, bar, pl.blocks, pl.per_group, pl.ppg,
                                          cooperative, s);
    if (e == hipSuccess) e = launch_set_step(const_cast<long long *>(c->geom.step_dev), n, 1, s);
    return e;
}
// reads the persistent launches' error flag (synchronises the stream)
int persistent_check(lbm_ctx *c, const char *what)
{
    unsigned err = 0;
    HIPCHK(c, hipMemcpyAsync(&err, c->ws + c->L.off_bar, sizeof(err), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (err) return fail(c, LBM_ESTATE, std::string(what) + ": a group barrier timed out (state invalid)");
    return LBM_OK;
}

// captured graphs hold the launch geometry: drop them when it changes
void drop_graphs(lbm_ctx *c)
{
    for (int p = 0; p < 2; ++p) {
        if (c->graph[p]) (void)hipGraphExecDestroy(c->graph[p]);
        if (c->pgraph[p]) (void)hipGraphExecDestroy(c->pgraph[p]);
        c->graph[p] = c->pgraph[p] = nullptr;
        c->graph_k[p] = c->pgraph_k[p] = 0;
    }
}

}  // namespace

extern "C" {

int lbm_describe(const lbm_config *cfg, lbm_layout *out)
{
    Layout L;
    const int rc = build_layout(cfg, L);
    if (rc != LBM_OK) return rc;
    if (out) {
        out->n_fluid_columns = L.ncol;
        out->plane_pitch = L.P;
        out->n_fluid_nodes = (int64_t)L.ncol * cfg->nz;
        out->state_bytes = (int64_t)L.state_bytes;
        out->workspace_bytes = (int64_t)L.total;
        out->bytes_per_update = 2 * 27 * (int64_t)L.elem;
        out->population_stride = L.pstride;
        out->record_bytes = (int64_t)L.record_bytes;
    }
    return LBM_OK;
}

int lbm_workspace_bytes(const lbm_config *cfg, size_t *bytes)
{
    Layout L;
    const int rc = build_layout(cfg, L);
    if (rc != LBM_OK) return rc;
    if (!bytes) return LBM_EINVAL;
    *bytes = L.total;
    return LBM_OK;
}

int lbm_init(const lbm_config *cfg, const double *amps, void *workspace, size_t bytes, void *stream, lbm_ctx **out)
{
    if (!out) return LBM_EINVAL;
    *out = nullptr;
    lbm_ctx *c = new (std::nothrow) lbm_ctx();
    if (!c) return LBM_ENOMEM;
    auto bail = [&](int rc) {
        delete c;
        return rc;
    };
    int rc = build_layout(cfg, c->L);
    if (rc != LBM_OK) return bail(rc);
    if (!workspace || bytes < c->L.total || ((uintptr_t)workspace & 255)) return bail(LBM_ENOMEM);
    if (cfg->n_modes > 0 && !amps) return bail(LBM_EINVAL);
    c->cfg = *cfg;
    c->ppl = cfg->batch;
    if (!c->cfg.block) c->cfg.block = c->L.step.block;
    if (!c->cfg.zchunk) c->cfg.zchunk = c->L.step.zchunk;
    c->stream = (hipStream_t)stream;
    c->ws = (char *)workspace;
    const lbm_config &g = c->cfg;
    const Layout &L = c->L;
    const size_t P = (size_t)L.P, B = (size_t)g.batch;

    // neighbour table: column of (x+dx, y+dy), periodic wrap, -1 if solid
    std::vector<int> nbr(9 * P, -1);
    std::vector<unsigned> colxy(P, 0xffffffffu);
    for (int k = 0; k < L.ncol; ++k) {
        colxy[k] = (unsigned)L.colx[k] | ((unsigned)L.coly[k] << 16);
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const int x = (L.colx[k] + dx + g.nx) % g.nx, y = (L.coly[k] + dy + g.ny) % g.ny;
                nbr[(size_t)((dy + 1) * 3 + (dx + 1)) * P + k] = L.colmap[(size_t)y * g.nx + x];
            }
    }
    std::vector<double> bcoef(g.wall == 1 ? 9 * P : 0, 0.0);
    if (g.wall == 1)
        for (int k = 0; k < L.ncol; ++k)
            for (int d = 0; d < 9; ++d)
                if (nbr[(size_t)d * P + k] < 0) {
                    const int dx = d % 3 - 1, dy = d / 3 - 1;
                    const bool far_fluid = nbr[(size_t)(8 - d) * P + k] >= 0;
                    bcoef[(size_t)d * P + k] = wall_coefficient(g, L.colx[k], L.coly[k], dx, dy, far_fluid);
                }
    // trigger-force shape sums per pipe and per column, Eq. (TurbForce)
    std::vector<float> fshape(B * 3 * P, 0.f);
    std::vector<double> fshape64(B * 3 * P, 0.0);
    std::vector<double> modes((size_t)2 * kMaxModes * 3 * P, 0.0);
    for (int k = 0; k < L.ncol; ++k)
        for (int q = 0; q < 2 * g.n_modes; ++q) {
            const int m = q / 2 + 1;
            const double phi = (q % 2) ? M_PI / (2.0 * m) : 0.0;
            double s[3];
            mode_shape(g, 1.0, m, phi, L.colx[k], L.coly[k], s);
            for (int d = 0; d < 3; ++d) modes[((size_t)q * 3 + d) * P + k] = s[d];
        }
    for (size_t b = 0; b < B; ++b)
        for (int k = 0; k < L.ncol; ++k)
            for (int d = 0; d < 3; ++d) {
                double v = 0.0;
                for (int q = 0; q < 2 * g.n_modes; ++q) v += amps[b * 2 * g.n_modes + q] * modes[((size_t)q * 3 + d) * P + k];
                fshape[(b * 3 + d) * P + k] = (float)v;
                fshape64[(b * 3 + d) * P + k] = v;
            }
    std::vector<float> ztab(2 * (size_t)g.nz);
    std::vector<double> ztab64(2 * (size_t)g.nz);
    for (int z = 0; z < g.nz; ++z) {
        const double ph = g.kz * 2.0 * M_PI * z / (double)g.nz;
        ztab64[z] = std::cos(ph);
        ztab64[g.nz + z] = std::sin(ph);
        ztab[z] = (float)ztab64[z];
        ztab[g.nz + z] = (float)ztab64[g.nz + z];
    }
    std::vector<float> sig((size_t)L.n_sigma);
    std::vector<double> sig64(g.storage == 2 ? (size_t)L.n_sigma : 0);
    for (long long n = 0; n < L.n_sigma; ++n) {
        const double v = std::sin(2.0 * M_PI * (double)n / g.period);
        sig[n] = (float)v;
        if (g.storage == 2) sig64[n] = v;
    }
    std::vector<double> u0(P, 0.0);
    if (g.init == 1)
        for (int k = 0; k < L.ncol; ++k) {
            const double dx = L.colx[k] - 0.5 * (g.nx - 1), dy = L.coly[k] - 0.5 * (g.ny - 1);
            u0[k] = loglaw(g, std::sqrt(dx * dx + dy * dy));
        }

    // FP16 references: E_c = fp32(32/27 d_c(u0)), c_z = 0, +1, -1, with the
    // per-axis equilibrium factors d_0 = -3/2 u^2, d_+-1 = +-3 u + 3 u^2 at the
    // column's initial velocity (the initial state is f^eq = w (1 + d_c(u0)))
    std::vector<float> href(g.storage == 1 ? 3 * P : 0, 0.f);
    if (g.storage == 1)
        for (int k = 0; k < L.ncol; ++k) {
            const double u = u0[k], f = 32.0 / 27.0;
            href[k] = (float)(f * (-1.5 * u * u));
            href[P + k] = (float)(f * (3.0 * u + 3.0 * u * u));
            href[2 * P + k] = (float)(f * (-3.0 * u + 3.0 * u * u));
        }

    char *ws = c->ws;
    auto h2d = [&](size_t off, const void *src, size_t n) {
        return n ? hipMemcpyAsync(ws + off, src, n, hipMemcpyHostToDevice, c->stream) : hipSuccess;
    };
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    double *scratch_dev = nullptr;  // set up the context-free entry point's scratch on this device
    if (e == hipSuccess) e = static_scratch(&scratch_dev);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = h2d(L.off_nbr, nbr.data(), nbr.size() * sizeof(int));
    if (e == hipSuccess) e = h2d(L.off_box, L.box.data(), L.box.size() * sizeof(int));
    if (e == hipSuccess) e = h2d(L.off_colxy, colxy.data(), colxy.size() * sizeof(unsigned));
    if (e == hipSuccess && g.wall == 1) e = h2d(L.off_bcoef, bcoef.data(), bcoef.size() * sizeof(double));
    if (e == hipSuccess) e = h2d(L.off_fshape, fshape.data(), fshape.size() * sizeof(float));
    if (e == hipSuccess) e = h2d(L.off_ztab, ztab.data(), ztab.size() * sizeof(float));
    if (e == hipSuccess) e = h2d(L.off_sigma, sig.data(), sig.size() * sizeof(float));
    if (e == hipSuccess) e = h2d(L.off_u0, u0.data(), u0.size() * sizeof(double));
    if (e == hipSuccess && g.storage == 2) e = h2d(L.off_fshape64, fshape64.data(), fshape64.size() * sizeof(double));
    if (e == hipSuccess && g.storage == 2) e = h2d(L.off_ztab64, ztab64.data(), ztab64.size() * sizeof(double));
    if (e == hipSuccess && g.storage == 2) e = h2d(L.off_sigma64, sig64.data(), sig64.size() * sizeof(double));
    if (e == hipSuccess && g.adjoint) e = h2d(L.off_modes, modes.data(), modes.size() * sizeof(double));
    if (e == hipSuccess && g.storage == 1) e = h2d(L.off_href, href.data(), href.size() * sizeof(float));
    if (e != hipSuccess) {
        std::fprintf(stderr, "lbm_init: %s\n", hipGetErrorString(e));
        if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
        return bail(LBM_EHIP);
    }

    Geom &G = c->geom;
    G.ncol = L.ncol;
    G.P = L.P;
    G.nx = g.nx;
    G.ny = g.ny;
    G.nz = g.nz;
    G.B = g.batch;
    G.pstride = (int)L.pstride;
    G.pipe = 27 * L.pstride;
    G.nbr = (const int *)(ws + L.off_nbr);
    G.bcoef = g.wall == 1 ? (const double *)(ws + L.off_bcoef) : nullptr;
    G.colxy = (const unsigned *)(ws + L.off_colxy);
    G.fshape = (const float *)(ws + L.off_fshape);
    G.ztab = (const float *)(ws + L.off_ztab);
    G.sigma = (const float *)(ws + L.off_sigma);
    G.n_sigma = L.n_sigma;
    G.step_dev = (const long long *)(ws + L.off_step);
    G.omega = (float)(1.0 / g.tau);
    c->t2 = Tiles2{L.nt2, kDefaultZChunk2, (g.nz + kDefaultZChunk2 - 1) / kDefaultZChunk2, 1, 0, g.batch,
                   (const int *)(ws + L.off_box)};
    G.accel_z = (float)g.accel_z;
    G.omega64 = 1.0 / g.tau;
    G.accel_z64 = g.accel_z;
    G.fshape64 = g.storage == 2 ? (const double *)(ws + L.off_fshape64) : nullptr;
    G.ztab64 = g.storage == 2 ? (const double *)(ws + L.off_ztab64) : nullptr;
    G.sigma64 = g.storage == 2 ? (const double *)(ws + L.off_sigma64) : nullptr;
    G.kind = 2 * g.collision + g.equilibrium;
    G.href = g.storage == 1 ? (const float *)(ws + L.off_href) : nullptr;
    G.check = (unsigned *)(ws + L.off_check);

    c->step = 0;
    e = launch_set_step((long long *)(ws + L.off_step), 0, 0, c->stream);
    if (e == hipSuccess) e = launch_fill(ws + L.off_check, sizeof(unsigned), c->stream);
    if (e == hipSuccess) e = launch_fill(ws + L.off_state[0], L.state_bytes, c->stream);  // padding reads as 0
    if (e == hipSuccess && L.off_state[1] != L.off_state[0]) e = launch_fill(ws + L.off_state[1], L.state_bytes, c->stream);
    if (e == hipSuccess) e = launch_fill(ws + L.off_prof_acc, B * P * 5 * sizeof(double), c->stream);
    if (e == hipSuccess) e = launch_init(g.storage, c->form(0), G, (const double *)(ws + L.off_u0), c->state(0), c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        std::fprintf(stderr, "lbm_init: %s\n", hipGetErrorString(e));
        (void)hipStreamDestroy(c->cap_stream);
        return bail(LBM_EHIP);
    }
    *out = c;
    return LBM_OK;
}

int lbm_step(lbm_ctx *c, int32_t n)
{
    CHECK_CTX(c);
    if (n < 0) return fail(c, LBM_EINVAL, "lbm_step: n must be >= 0");
    return do_step_eager(c, n);
}

int lbm_step_graph(lbm_ctx *c, int32_t n, int32_t k)
{
    CHECK_CTX(c);
    if (n < 0 || k < 2 || k > 1024 || (k & 1)) return fail(c, LBM_EINVAL, "lbm_step_graph: need n >= 0, even k in 2..1024");
    if (n >= k) {
        // one graph per starting buffer: with an odd number of two-step
        // launches per graph, consecutive replays alternate between them
        const int reps = n / k;
        for (int r = 0; r < reps; ++r) {
            const int par = c->buf(c->step);
            if (!c->graph[par] || c->graph_k[par] != k) {
                if (c->graph[par]) {
                    (void)hipGraphExecDestroy(c->graph[par]);
                    c->graph[par] = nullptr;
                }
                hipGraph_t gr = nullptr;
                HIPCHK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
                hipError_t e = launch_steps(c, c->step, k, c->flip, c->cap_stream);
                if (e == hipSuccess) e = launch_set_step(const_cast<long long *>(c->geom.step_dev), k, 1, c->cap_stream);
                const hipError_t e2 = hipStreamEndCapture(c->cap_stream, &gr);
                if (e != hipSuccess || e2 != hipSuccess) {
                    if (gr) (void)hipGraphDestroy(gr);
                    return fail(c, LBM_EHIP, std::string("graph capture failed: ") +
                                                 hipGetErrorString(e != hipSuccess ? e : e2));
                }
                hipGraphExec_t ex = nullptr;
                const hipError_t e3 = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
                (void)hipGraphDestroy(gr);
                if (e3 != hipSuccess) return fail(c, LBM_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e3));
                c->graph[par] = ex;
                c->graph_k[par] = k;
            }
            HIPCHK(c, hipGraphLaunch(c->graph[par], c->stream));
            c->flip = flip_after(c, k);
            c->step += k;
        }
        n -= reps * k;
    }
    return do_step_eager(c, n);
}

int lbm_step_persistent(lbm_ctx *c, int32_t n)
{
    CHECK_CTX(c);
    if (n < 0) return fail(c, LBM_EINVAL, "lbm_step_persistent: n must be >= 0");
    if (n == 0) return LBM_OK;
    PersistentPlan pl;
    int rc = persistent_plan(c, pl);
    if (rc != LBM_OK) return rc;
    unsigned *bar = (unsigned *)(c->ws + c->L.off_bar);
    HIPCHK(c, launch_fill(bar, 32 * sizeof(unsigned) * ((size_t)pl.groups + 1), c->stream));
    HIPCHK(c, launch_persistent(c, pl, n, 1, c->stream));
    c->step += n;
    return persistent_check(c, "lbm_step_persistent");
}

int lbm_step_persistent_graph(lbm_ctx *c, int32_t n, int32_t k)
{
    CHECK_CTX(c);
    if (n < 0 || k < 2 || k > (1 << 20) || (k & 1))
        return fail(c, LBM_EINVAL, "lbm_step_persistent_graph: need n >= 0, even k in 2..2^20");
    PersistentPlan pl;
    int rc = persistent_plan(c, pl);
    if (rc != LBM_OK) return rc;
    unsigned *bar = (unsigned *)(c->ws + c->L.off_bar);
    const int reps = n / k;
    if (reps > 0) {
        HIPCHK(c, launch_fill(bar, 32 * sizeof(unsigned), c->stream));  // the error flag, once for all replays
        for (int r = 0; r < reps; ++r) {
            const int par = c->buf(c->step);  // k is even: a replay ends in the buffer it starts from
            if (!c->pgraph[par] || c->pgraph_k[par] != k) {
                if (c->pgraph[par]) {
                    (void)hipGraphExecDestroy(c->pgraph[par]);
                    c->pgraph[par] = nullptr;
                }
                hipGraph_t gr = nullptr;
                HIPCHK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
                // group counters and barriers (the error flag stays), one
                // persistent launch of k steps, the step counter
                hipError_t e = launch_fill(bar + 32, 32 * sizeof(unsigned) * (size_t)pl.groups, c->cap_stream);
                if (e == hipSuccess) e = launch_persistent(c, pl, k, 0, c->cap_stream);
                const hipError_t e2 = hipStreamEndCapture(c->cap_stream, &gr);
                if (e != hipSuccess || e2 != hipSuccess) {
                    if (gr) (void)hipGraphDestroy(gr);
                    return fail(c, LBM_EHIP, std::string("persistent graph capture failed: ") +
                                                 hipGetErrorString(e != hipSuccess ? e : e2));
                }
                hipGraphExec_t ex = nullptr;
                const hipError_t e3 = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
                (void)hipGraphDestroy(gr);
                if (e3 != hipSuccess) return fail(c, LBM_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e3));
                c->pgraph[par] = ex;
                c->pgraph_k[par] = k;
            }
            HIPCHK(c, hipGraphLaunch(c->pgraph[par], c->stream));
            c->step += k;
        }
        rc = persistent_check(c, "lbm_step_persistent_graph");
        if (rc != LBM_OK) return rc;
    }
    return n % k ? lbm_step_persistent(c, n % k) : LBM_OK;
}

int lbm_set_launch(lbm_ctx *c, int32_t block, int32_t zchunk, int32_t xcd_remap, int32_t ppl, int32_t pipe_major)
{
    CHECK_CTX(c);
    if (pipe_major < -1 || pipe_major > 1) return fail(c, LBM_EINVAL, "pipe_major must be -1, 0 or 1");
    if (block && block != 64 && block != 128 && block != 256 && block != 512)
        return fail(c, LBM_EINVAL, "block must be 64, 128, 256 or 512");
    if (zchunk && (zchunk < 1 || zchunk > 64)) return fail(c, LBM_EINVAL, "zchunk must be in 1..64");
    if (xcd_remap < -1 || xcd_remap > 4096) return fail(c, LBM_EINVAL, "xcd_remap must be in -1..4096");
    if (ppl < 0 || ppl > c->cfg.batch) return fail(c, LBM_EINVAL, "pipes_per_launch must be in 0..batch");
    Tiles &t = c->L.step;
    if (block) {
        t.block = block;
        t.nkb = (c->L.ncol + block - 1) / block;
        c->cfg.block = block;
    }
    if (zchunk) {
        t.zchunk = zchunk;
        t.nzc = (c->cfg.nz + zchunk - 1) / zchunk;
        c->cfg.zchunk = zchunk;
    }
    if (xcd_remap >= 0) {
        t.xcd = xcd_remap;
        c->cfg.xcd_remap = xcd_remap;
    }
    if (ppl) c->ppl = ppl;
    if (pipe_major >= 0) c->pipe_major = pipe_major;
    drop_graphs(c);
    return LBM_OK;
}

int lbm_set_fused(lbm_ctx *c, int32_t steps_per_launch, int32_t zchunk, int32_t xcd_remap)
{
    CHECK_CTX(c);
    if (steps_per_launch < 0 || steps_per_launch > 2) return fail(c, LBM_EINVAL, "steps_per_launch must be 0, 1 or 2");
    if (steps_per_launch == 2 && !c->can_fuse())
        return fail(c, LBM_EINVAL, "two steps per launch need the two-buffer pattern, the halfway bounce-back wall, "
                                   "FP32 or FP16 storage and the paper's collision");
    if (zchunk < 0 || zchunk > 1024) return fail(c, LBM_EINVAL, "zchunk must be in 0..1024");
    if (xcd_remap < -1 || xcd_remap > 4096) return fail(c, LBM_EINVAL, "xcd_remap must be in -1..4096");
    if (steps_per_launch) c->fuse = steps_per_launch;
    if (zchunk) {
        c->t2.zchunk = zchunk;
        c->t2.nzc = (c->cfg.nz + zchunk - 1) / zchunk;
    }
    if (xcd_remap >= 0) c->t2.xcd = xcd_remap;
    drop_graphs(c);
    return LBM_OK;
}

int lbm_stream_copy(lbm_ctx *c, int32_t n)
{
    CHECK_CTX(c);
    if (n < 0) return fail(c, LBM_EINVAL, "lbm_stream_copy: n must be >= 0");
    for (int j = 0; j < n; ++j)
        HIPCHK(c, launch_stream_copy(c->cfg.storage, c->geom, c->L.step, c->state(c->step), c->state(c->step + 1),
                                     c->stream));
    return LBM_OK;
}

int lbm_get_step(const lbm_ctx *c, int64_t *step)
{
    if (!c || !step) return LBM_EINVAL;
    *step = c->step;
    return LBM_OK;
}

int lbm_moments(lbm_ctx *c, float *rho, float *u)
{
    CHECK_CTX(c);
    if (!rho && !u) return LBM_OK;
    const size_t nodes = (size_t)c->cfg.batch * c->cfg.nz * c->cfg.ny * c->cfg.nx;
    if (rho) HIPCHK(c, launch_fill(rho, nodes * sizeof(float), c->stream));
    if (u) HIPCHK(c, launch_fill(u, 3 * nodes * sizeof(float), c->stream));
    ObserveArgs o{};
    o.flags = OBS_MOMENTS;
    o.rho = rho;
    o.u = u;
    return observe(c, o);
}

int lbm_populations(lbm_ctx *c, float *g)
{
    CHECK_CTX(c);
    if (!g) return fail(c, LBM_EINVAL, "lbm_populations: NULL output");
    const size_t nodes = (size_t)c->cfg.batch * c->cfg.nz * c->cfg.ny * c->cfg.nx;
    HIPCHK(c, launch_fill(g, 27 * nodes * sizeof(float), c->stream));
    ObserveArgs o{};
    o.flags = OBS_POPS;
    o.pops = g;
    return observe(c, o);
}

int lbm_set_populations(lbm_ctx *c, const float *g, int64_t step)
{
    CHECK_CTX(c);
    if (!g || step < 0) return fail(c, LBM_EINVAL, "lbm_set_populations: NULL input or negative step");
    c->step = step;
    c->mass_ref.clear();
    HIPCHK(c, launch_set_pops(c->cfg.storage, c->form(step), c->geom, g, c->state(step), c->stream));
    HIPCHK(c, launch_set_step(const_cast<long long *>(c->geom.step_dev), step, 0, c->stream));
    return LBM_OK;
}

int lbm_check_flags(lbm_ctx *c, uint32_t *flags, int32_t *checked)
{
    CHECK_CTX(c);
    if (!flags) return fail(c, LBM_EINVAL, "lbm_check_flags: NULL output");
    unsigned v = 0;
    HIPCHK(c, hipMemcpyAsync(&v, c->ws + c->L.off_check, sizeof(v), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    *flags = v;
    if (checked) *checked = LBM_CHECKED;
    return LBM_OK;
}

int lbm_diagnostics(lbm_ctx *c, double *host_out)
{
    CHECK_CTX(c);
    if (!host_out) return fail(c, LBM_EINVAL, "lbm_diagnostics: NULL output");
    ObserveArgs o{};
    o.flags = OBS_DIAG;
    o.diag_part = (double *)(c->ws + c->L.off_diag_part);
    int rc = observe(c, o);
    if (rc != LBM_OK) return rc;
    double *dout = (double *)(c->ws + c->L.off_diag_out);
    HIPCHK(c, launch_reduce_diag(c->geom, c->L.obs, o.diag_part, dout, c->stream));
    HIPCHK(c, hipMemcpyAsync(host_out, dout, (size_t)c->cfg.batch * 5 * sizeof(double), hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int b = 0; b < c->cfg.batch; ++b)
        if (host_out[b * 5 + 4] != 0.0 || !std::isfinite(host_out[b * 5])) return fail(c, LBM_ENAN, "non-finite populations");
    if (c->watch_tol > 0.0) {
        if (c->mass_ref.empty()) {
            c->mass_ref.resize(c->cfg.batch);
            for (int b = 0; b < c->cfg.batch; ++b) c->mass_ref[b] = host_out[b * 5];
        } else {
            for (int b = 0; b < c->cfg.batch; ++b) {
                const double drift = std::fabs(host_out[b * 5] - c->mass_ref[b]) / std::fabs(c->mass_ref[b]);
                if (!(drift <= c->watch_tol)) {
                    char buf[160];
                    std::snprintf(buf, sizeof buf, "mass drift of pipe %d: %.3e relative (limit %.3e)", b, drift,
                                  c->watch_tol);
                    return fail(c, LBM_ENAN, buf);
                }
            }
        }
    }
    return LBM_OK;
}

int lbm_set_watchdog(lbm_ctx *c, double mass_rel_tol)
{
    CHECK_CTX(c);
    if (!(mass_rel_tol >= 0.0) || !std::isfinite(mass_rel_tol))
        return fail(c, LBM_EINVAL, "lbm_set_watchdog: the limit must be finite and >= 0");
    c->watch_tol = mass_rel_tol;
    c->mass_ref.clear();
    return LBM_OK;
}

int lbm_energy(lbm_ctx *c, double *host_out)
{
    CHECK_CTX(c);
    if (!host_out) return fail(c, LBM_EINVAL, "lbm_energy: NULL output");
    ObserveArgs o{};
    o.flags = OBS_ENERGY;
    o.energy_part = (double *)(c->ws + c->L.off_energy_part);
    int rc = observe(c, o);
    if (rc != LBM_OK) return rc;
    double *eout = (double *)(c->ws + c->L.off_energy_out);
    HIPCHK(c, launch_reduce_energy(c->geom, c->L.obs, o.energy_part, eout, c->stream));
    HIPCHK(c, hipMemcpyAsync(host_out, eout, (size_t)c->cfg.batch * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const double nf = (double)c->L.ncol * c->cfg.nz;
    for (int b = 0; b < c->cfg.batch; ++b) host_out[b] /= nf;
    return LBM_OK;
}

int lbm_energy_accumulate(lbm_ctx *c, double *acc)
{
    CHECK_CTX(c);
    if (!acc) return fail(c, LBM_EINVAL, "lbm_energy_accumulate: NULL accumulator");
    ObserveArgs o{};
    o.flags = OBS_ENERGY;
    o.energy_part = (double *)(c->ws + c->L.off_energy_part);
    int rc = observe(c, o);
    if (rc != LBM_OK) return rc;
    const double nf = (double)c->L.ncol * c->cfg.nz;
    HIPCHK(c, launch_accumulate_energy(c->geom, c->L.obs, o.energy_part, 1.0 / nf, acc, c->stream));
    return LBM_OK;
}

int lbm_recompute(lbm_ctx *c, const void *start, int64_t s0, int32_t n, void *ring, size_t stride)
{
    CHECK_CTX(c);
    if (!start || !ring || n < 1 || s0 < 0) return fail(c, LBM_EINVAL, "lbm_recompute: bad arguments");
    if (c->cfg.pattern != 0) return fail(c, LBM_EINVAL, "lbm_recompute needs the two-buffer pattern");
    if (stride < c->L.state_bytes || (stride & 255) || ((uintptr_t)ring & 255))
        return fail(c, LBM_EINVAL, "lbm_recompute: stride must be >= the state size and ring/stride 256-byte aligned");
    char *r = (char *)ring;
    if (start != ring) HIPCHK(c, hipMemcpyAsync(r, start, c->L.state_bytes, hipMemcpyDeviceToDevice, c->stream));
    if (n == 1) return LBM_OK;
    Geom g = c->geom;
    g.step_dev = (const long long *)(c->ws + c->L.off_step2);
    HIPCHK(c, launch_set_step((long long *)(c->ws + c->L.off_step2), s0, 0, c->stream));
    Tiles t = c->L.step;
    t.b0 = 0;
    t.nb = c->cfg.batch;
    for (int j = 0; j + 1 < n; ++j)
        HIPCHK(c, launch_step(c->cfg.storage, g, t, r + (size_t)j * stride, r + (size_t)(j + 1) * stride, j, c->stream));
    return LBM_OK;
}

int lbm_step_recording(lbm_ctx *c, int32_t n, void *records, size_t record_stride)
{
    CHECK_CTX(c);
    if (n < 0 || (n > 0 && !records)) return fail(c, LBM_EINVAL, "lbm_step_recording: bad arguments");
    if (c->cfg.pattern != 0 || c->fuse != 1)
        return fail(c, LBM_EINVAL, "lbm_step_recording needs the two-buffer pattern and one step per launch");
    if (c->cfg.collision != 0 || c->cfg.equilibrium != 0)
        return fail(c, LBM_EINVAL, "lbm_step_recording: the paper's scheme only (collision = equilibrium = 0)");
    if (record_stride < c->L.record_bytes || (record_stride & 255) || ((uintptr_t)records & 255))
        return fail(c, LBM_EINVAL, "lbm_step_recording: record stride below the record size or not 256-byte aligned");
    if (n == 0) return LBM_OK;
    Tiles t = c->L.step;
    t.b0 = 0;
    t.nb = c->cfg.batch;
    char *r = (char *)records;
    for (int j = 0; j < n; ++j) {
        const int bi = (int)((c->step + j + c->flip) & 1);
        HIPCHK(c, launch_step_record(c->cfg.storage, c->geom, t, c->ws + c->L.off_state[bi],
                                     c->ws + c->L.off_state[bi ^ 1], j, r + (size_t)j * record_stride, c->stream));
    }
    HIPCHK(c, launch_set_step(const_cast<long long *>(c->geom.step_dev), n, 1, c->stream));
    c->step += n;
    return LBM_OK;
}

int lbm_recompute_moments(lbm_ctx *c, const void *start, int64_t s0, int32_t n, void *scratch, size_t stride,
                          void *records, size_t record_stride)
{
    CHECK_CTX(c);
    if (!start || !scratch || !records || n < 1 || s0 < 0)
        return fail(c, LBM_EINVAL, "lbm_recompute_moments: bad arguments");
    if (c->cfg.pattern != 0) return fail(c, LBM_EINVAL, "lbm_recompute_moments needs the two-buffer pattern");
    if (c->cfg.collision != 0 || c->cfg.equilibrium != 0)
        return fail(c, LBM_EINVAL, "lbm_recompute_moments: the paper's scheme only (collision = equilibrium = 0)");
    if (stride < c->L.state_bytes || (stride & 255) || ((uintptr_t)scratch & 255) ||
        record_stride < c->L.record_bytes || (record_stride & 255) || ((uintptr_t)records & 255))
        return fail(c, LBM_EINVAL, "lbm_recompute_moments: strides below the state / record size or not 256-byte "
                                   "aligned");
    const char *st = (const char *)start;
    char *s = (char *)scratch, *r = (char *)records;
    // start is scratch state 0 itself or lies outside both scratch states
    const size_t sb = c->L.state_bytes;
    if (st != s && st < s + stride + sb && st + sb > s)
        return fail(c, LBM_EINVAL, "lbm_recompute_moments: start overlaps the scratch states");
    if (st != s) HIPCHK(c, hipMemcpyAsync(s, start, c->L.state_bytes, hipMemcpyDeviceToDevice, c->stream));
    Geom g = c->geom;
    g.step_dev = (const long long *)(c->ws + c->L.off_step2);
    HIPCHK(c, launch_set_step((long long *)(c->ws + c->L.off_step2), s0, 0, c->stream));
    Tiles t = c->L.step;
    t.b0 = 0;
    t.nb = c->cfg.batch;
    for (int j = 0; j < n; ++j)
        HIPCHK(c, launch_step_record(c->cfg.storage, g, t, s + (size_t)(j & 1) * stride,
                                     s + (size_t)((j + 1) & 1) * stride, j, r + (size_t)j * record_stride, c->stream));
    return LBM_OK;
}

int lbm_profile_accumulate(lbm_ctx *c)
{
    CHECK_CTX(c);
    ObserveArgs o{};
    o.flags = OBS_PROFILE;
    o.prof_part = (double *)(c->ws + c->L.off_prof_part);
    int rc = observe(c, o);
    if (rc != LBM_OK) return rc;
    HIPCHK(c, launch_reduce_profile(c->geom, c->L.obs, o.prof_part, (double *)(c->ws + c->L.off_prof_acc), c->stream));
    return LBM_OK;
}

int lbm_profile_reset(lbm_ctx *c)
{
    CHECK_CTX(c);
    HIPCHK(c, launch_fill(c->ws + c->L.off_prof_acc, (size_t)c->cfg.batch * c->L.P * 5 * sizeof(double), c->stream));
    return LBM_OK;
}

int lbm_profile_read(lbm_ctx *c, double *host_out)
{
    CHECK_CTX(c);
    if (!host_out) return fail(c, LBM_EINVAL, "lbm_profile_read: NULL output");
    const size_t P = (size_t)c->L.P, B = (size_t)c->cfg.batch;
    std::vector<double> acc(B * P * 5);
    HIPCHK(c, hipMemcpyAsync(acc.data(), c->ws + c->L.off_prof_acc, acc.size() * sizeof(double), hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const size_t plane = (size_t)c->cfg.nx * c->cfg.ny;
    std::memset(host_out, 0, B * plane * 5 * sizeof(double));
    for (size_t b = 0; b < B; ++b)
        for (int k = 0; k < c->L.ncol; ++k) {
            const size_t cell = (size_t)c->L.coly[k] * c->cfg.nx + c->L.colx[k];
            for (int q = 0; q < 5; ++q) host_out[(b * plane + cell) * 5 + q] = acc[(b * P + k) * 5 + q];
        }
    return LBM_OK;
}

int lbm_state_bytes(const lbm_ctx *c, size_t *bytes)
{
    if (!c || !bytes) return LBM_EINVAL;
    *bytes = c->L.state_bytes;
    return LBM_OK;
}

int lbm_save(lbm_ctx *c, void *dst, int64_t *step)
{
    CHECK_CTX(c);
    if (!dst) return fail(c, LBM_EINVAL, "lbm_save: NULL destination");
    HIPCHK(c, hipMemcpyAsync(dst, c->state(c->step), c->L.state_bytes, hipMemcpyDeviceToDevice, c->stream));
    if (step) *step = c->step;
    return LBM_OK;
}

int lbm_load(lbm_ctx *c, const void *src, int64_t step)
{
    CHECK_CTX(c);
    if (!src || step < 0) return fail(c, LBM_EINVAL, "lbm_load: NULL source or negative step");
    c->step = step;
    c->mass_ref.clear();
    HIPCHK(c, hipMemcpyAsync(c->state(step), src, c->L.state_bytes, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, launch_set_step(const_cast<long long *>(c->geom.step_dev), step, 0, c->stream));
    return LBM_OK;
}

int lbm_adjoint_reset(lbm_ctx *c, int64_t obs_begin, int64_t obs_end)
{
    CHECK_CTX(c);
    if (!c->cfg.adjoint) return fail(c, LBM_ESTATE, "adjoint buffers absent (cfg.adjoint == 0)");
    if (obs_begin < 0 || obs_end <= obs_begin) return fail(c, LBM_EINVAL, "need 0 <= obs_begin < obs_end");
    c->obs_begin = obs_begin;
    c->obs_end = obs_end;
    c->cursor = obs_end - 1;
    c->lam_cur = 0;
    c->adj_ready = true;
    const size_t lam = (size_t)c->geom.pipe * c->cfg.batch * (c->cfg.adjoint == 2 ? sizeof(double) : sizeof(float));
    HIPCHK(c, launch_fill(c->ws + c->L.off_lam[0], lam, c->stream));
    HIPCHK(c, launch_fill(c->ws + c->L.off_lam[1], lam, c->stream));
    HIPCHK(c, launch_fill(c->ws + c->L.off_grad_col, (size_t)c->cfg.batch * c->L.P * 3 * sizeof(double), c->stream));
    HIPCHK(c, launch_fill(c->ws + c->L.off_grad_part, (size_t)c->cfg.batch * c->L.adj.nzc * c->L.P * 3 * sizeof(double),
                          c->stream));
    c->grad_base_set = false;
    return LBM_OK;
}

// n reverse steps from saved states (records == false) or moment records
static int adjoint_sweep(lbm_ctx *c, int32_t n, const void *fwd, size_t stride, bool records, double *grad)
{
    const char *name = records ? "lbm_adjoint_step_moments" : "lbm_adjoint_step";
    char msg[160];
    if (!c->cfg.adjoint || !c->adj_ready) {
        std::snprintf(msg, sizeof msg, "%s before lbm_adjoint_reset", name);
        return fail(c, LBM_ESTATE, msg);
    }
    if (n < 1 || !fwd || (c->cfg.n_modes > 0 && !grad)) {
        std::snprintf(msg, sizeof msg, "%s: bad arguments", name);
        return fail(c, LBM_EINVAL, msg);
    }
    if (c->cursor - n + 1 < 0) {
        std::snprintf(msg, sizeof msg, "%s: cursor would move below 0", name);
        return fail(c, LBM_ESTATE, msg);
    }
    if (stride < (records ? c->L.record_bytes : c->L.state_bytes)) {
        std::snprintf(msg, sizeof msg, "%s: stride < %s size", name, records ? "record" : "state");
        return fail(c, LBM_EINVAL, msg);
    }
    const int nq = 2 * c->cfg.n_modes;
    const double wgt = 1.0 / ((double)(c->obs_end - c->obs_begin) * (double)c->L.ncol * c->cfg.nz);
    double *acc = (double *)(c->ws + c->L.off_grad_col), *base = (double *)(c->ws + c->L.off_grad_base);
    if (nq > 0 && !c->grad_base_set) {
        HIPCHK(c, hipMemcpyAsync(base, grad, (size_t)c->cfg.batch * nq * sizeof(double), hipMemcpyDeviceToDevice,
                                 c->stream));
        c->grad_base_set = true;
    }
    for (int j = n - 1; j >= 0; --j) {
        AdjointArgs a{};
        (records ? a.rec : a.state) = (const char *)fwd + (size_t)j * stride;
        a.lam_in = c->ws + c->L.off_lam[c->lam_cur];
        a.lam_out = c->ws + c->L.off_lam[c->lam_cur ^ 1];
        a.grad_part = (double *)(c->ws + c->L.off_grad_part);
        a.cursor = c->cursor;
        a.in_window = c->cursor >= c->obs_begin && c->cursor < c->obs_end;
        a.has_next = c->cursor + 1 < c->obs_end;
        a.energy_weight = wgt;
        // (the kernel adds sigma(c) times its sensitivities to the partials)
        HIPCHK(c, launch_adjoint(c->cfg.storage, c->cfg.adjoint, c->geom, c->L.adj, a, c->stream));
        c->lam_cur ^= 1;
        c->cursor -= 1;
    }
    if (nq > 0) {
        HIPCHK(c, launch_grad_accumulate(c->geom, c->L.adj, (const double *)(c->ws + c->L.off_grad_part), acc,
                                         c->stream));
        HIPCHK(c, launch_project_grad(c->geom, acc, (const double *)(c->ws + c->L.off_modes), nq, base, grad, c->stream));
    }
    return LBM_OK;
}

int lbm_adjoint_step(lbm_ctx *c, int32_t n, const void *fwd_states, size_t state_stride, double *grad)
{
    CHECK_CTX(c);
    return adjoint_sweep(c, n, fwd_states, state_stride, false, grad);
}

int lbm_adjoint_step_moments(lbm_ctx *c, int32_t n, const void *records, size_t record_stride, double *grad)
{
    CHECK_CTX(c);
    return adjoint_sweep(c, n, records, record_stride, true, grad);
}

int lbm_ring_sample(lbm_ctx *c, double r0, int32_t ntheta, float *ring)
{
    CHECK_CTX(c);
    if (!ring || ntheta < 4 || ntheta > kMaxRing || !(r0 > 0.0))
        return fail(c, LBM_EINVAL, "lbm_ring_sample: need ring != NULL, 4 <= ntheta <= 4096, r0 > 0");
    if (!(c->cfg.radius > 0.0)) return fail(c, LBM_EINVAL, "lbm_ring_sample: needs a pipe wall (radius > 0)");
    if (r0 != c->ring_r0 || ntheta != c->ring_n) {
        const int nx = c->cfg.nx, ny = c->cfg.ny;
        const double xc = 0.5 * (nx - 1), yc = 0.5 * (ny - 1);
        c->ring_nodes.clear();
        c->ring_idx.assign((size_t)ntheta * 4, 0);
        c->ring_w.assign((size_t)ntheta * 4, 0.0);
        std::vector<int> slot(c->L.ncol, -1);  // column -> index in ring_nodes
        for (int j = 0; j < ntheta; ++j) {
            const double th = 2.0 * M_PI * j / ntheta;
            const double px = xc + r0 * std::cos(th), py = yc + r0 * std::sin(th);
            const int x0 = (int)std::floor(px), y0 = (int)std::floor(py);
            const double fx = px - x0, fy = py - y0;
            const int xs[4] = {x0, x0 + 1, x0, x0 + 1}, ys[4] = {y0, y0, y0 + 1, y0 + 1};
            const double ws[4] = {(1 - fx) * (1 - fy), fx * (1 - fy), (1 - fx) * fy, fx * fy};
            for (int q = 0; q < 4; ++q) {
                const int col = (xs[q] >= 0 && xs[q] < nx && ys[q] >= 0 && ys[q] < ny)
                                    ? c->L.colmap[(size_t)ys[q] * nx + xs[q]] : -1;
                if (col < 0) {
                    c->ring_r0 = -1.0;
                    return fail(c, LBM_EINVAL, "lbm_ring_sample: the ring touches a solid node (r0 too large)");
                }
                if (slot[col] < 0) {
                    slot[col] = (int)c->ring_nodes.size();
                    c->ring_nodes.push_back(col);
                }
                c->ring_idx[(size_t)j * 4 + q] = slot[col];
                c->ring_w[(size_t)j * 4 + q] = ws[q];
            }
        }
        HIPCHK(c, hipMemcpyAsync(c->ws + c->L.off_ring_nodes, c->ring_nodes.data(),
                                 c->ring_nodes.size() * sizeof(int), hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(c->ws + c->L.off_ring_idx, c->ring_idx.data(), c->ring_idx.size() * sizeof(int),
                                 hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(c->ws + c->L.off_ring_w, c->ring_w.data(), c->ring_w.size() * sizeof(double),
                                 hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));  // the host tables may be rebuilt by the next call
        c->ring_r0 = r0;
        c->ring_n = ntheta;
    }
    const RingArgs r{(const int *)(c->ws + c->L.off_ring_nodes), (const int *)(c->ws + c->L.off_ring_idx),
                     (const double *)(c->ws + c->L.off_ring_w), (int)c->ring_nodes.size(), ntheta};
    HIPCHK(c, launch_ring(c->cfg.storage, c->form(c->step), c->geom, r, c->state(c->step), ring, c->stream));
    return LBM_OK;
}

int lbm_ring_spectrum(lbm_ctx *c, const float *ring, int32_t ntheta, int32_t mmax, double *spec, double *mean,
                      int32_t *dominant)
{
    CHECK_CTX(c);
    if (!ring || !spec || ntheta < 4 || ntheta > kMaxRing || mmax < 1 || mmax > ntheta / 2 || (dominant && !mean))
        return fail(c, LBM_EINVAL,
                    "lbm_ring_spectrum: need ring, spec != NULL, 4 <= ntheta <= 4096, 1 <= mmax <= ntheta/2, "
                    "mean when dominant is requested");
    if (ntheta != c->tw_n) {
        c->twiddle.assign((size_t)ntheta * 2, 0.0);
        for (int q = 0; q < ntheta; ++q) {
            const double a = 2.0 * M_PI * q / ntheta;
            c->twiddle[2 * q] = std::cos(a);
            c->twiddle[2 * q + 1] = -std::sin(a);
        }
        HIPCHK(c, hipMemcpyAsync(c->ws + c->L.off_twiddle, c->twiddle.data(), c->twiddle.size() * sizeof(double),
                                 hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        c->tw_n = ntheta;
    }
    HIPCHK(c, launch_ring_spectrum(ring, c->cfg.batch * c->cfg.nz, ntheta, mmax,
                                   (const double *)(c->ws + c->L.off_twiddle), spec, c->stream));
    if (mean) HIPCHK(c, launch_spectrum_mean(spec, c->cfg.batch, c->cfg.nz, mmax, mean, dominant, c->stream));
    return LBM_OK;
}

const char *lbm_last_error(const lbm_ctx *c)
{
    if (!c) return "no context";
    return c->err.c_str();
}

void lbm_destroy(lbm_ctx *c)
{
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    drop_graphs(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    delete c;
}

}  // extern "C"
