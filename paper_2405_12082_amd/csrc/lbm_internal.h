// lbm_internal.h -- kernel argument blocks and launchers shared by the
// runtime (lbm_runtime.hip) and the kernels (lbm_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// Checked builds (-DLBM_CHECKED=1, liblbm_checked.so): device-side bounds
// tests on the gather, store and table accesses (lbm_device.h), their
// violations reported by lbm_check_flags.  0: the release build.
#ifndef LBM_CHECKED
#define LBM_CHECKED 0
#endif

namespace lbm {

// z-invariant geometry and forcing tables, all in the caller's workspace
struct Geom {
    int ncol;        // fluid columns of one cross-section
    int P;           // plane pitch (elements), multiple of 64
    int nx, ny, nz, B;
    int pstride;     // elements between populations of one pipe (nz * P, padded)
    long long pipe;  // 27 * pstride: elements between pipes
    const int *nbr;          // [9][P]: column of (x+dx, y+dy), -1 if solid
    const unsigned *colxy;   // [P]: x | y << 16
    const float *fshape;     // [B][3][P]: trigger shape sums (P_x, P_y, Q)
    const float *ztab;       // [2][nz]: cos, sin(k_z 2 pi z / L)
    const float *sigma;      // [n_sigma]: sin(2 pi n / T) for n < force_off_step
    long long n_sigma;
    const long long *step_dev;  // device step counter (graph-safe)
    const double *bcoef;        // [9][P] interpolated-wall coefficients (see pull_one), null: bounce-back
    float omega, accel_z;
    // FP64 storage computes in FP64 throughout: its own copies of the force
    // tables and of omega and h (null / unused for FP32 and FP16 storage)
    const double *fshape64;  // [B][3][P]
    const double *ztab64;    // [2][nz]
    const double *sigma64;   // [n_sigma]
    double omega64, accel_z64;
    int kind;  // collision kind (CollisionKind): 0 the paper's MRT scheme, 1..3 comparison schemes
    // FP16 storage: per-column references [3][P], E_c = fp32(32/27 d_c(u0)) for
    // c_z = 0, +1, -1 (d_c the per-axis equilibrium factor at the column's
    // initial velocity u0); null for FP32 / FP64 storage
    const float *href;
    unsigned *check;  // checked builds: bounds-violation flags (CheckBit), one word
};

// tile decomposition of a launch: BLOCK consecutive columns x zchunk planes x pipe
struct Tiles {
    int block, zchunk, nkb, nzc;
    int xcd;  // nonzero: XCD-aware workgroup -> tile mapping
    int b0;   // first pipe of the launch
    int nb;   // pipes covered by the launch
    __host__ __device__ long long count() const { return (long long)nkb * nzc; }
};

// Two time steps per launch (temporal blocking): the cross-section is cut
// into 14 x 14 column tiles; a workgroup takes one tile, its ring of halo
// columns (a 16 x 16 box, one thread per box column) and a range of zchunk
// planes.  box[tile][slot] is the column of each box slot (periodic wrap),
// with FUSED_OWNED set on the tile's own interior columns, or -1 where the
// box slot is solid.
constexpr int FUSED_BX = 16, FUSED_BY = 16, FUSED_BOX = FUSED_BX * FUSED_BY;
constexpr int FUSED_IN = FUSED_BX - 2;  // interior columns per tile row
constexpr int FUSED_OWNED = 1 << 30;
struct Tiles2 {
    int nt;           // tiles with at least one owned fluid column
    int zchunk, nzc;  // output planes per workgroup, z-chunks
    int xcd;          // workgroup -> tile order, as Tiles::xcd
    int b0, nb;       // pipes covered by the launch
    const int *box;   // [nt][FUSED_BOX]
    __host__ __device__ long long count() const { return (long long)nt * nzc; }
};

// Forms of a population buffer between steps:
//  FORM_S: slot i of node y holds g*_i(y, n-1), the post-collision value that
//          node y + c_i pulls (two-buffer pattern);
//  FORM_W: the same with slots i and opp(i) exchanged (AA pattern, odd n);
//  FORM_N: slot i of node x holds g_i(x, n) itself (AA pattern, even n).
enum StateForm : int { FORM_S = 0, FORM_W = 1, FORM_N = 2 };

enum ObserveFlags {
    OBS_MOMENTS = 1,   // dense rho / u outputs
    OBS_POPS = 2,      // dense population deviations
    OBS_DIAG = 4,      // FP64 mass / momentum / non-finite partials per tile
    OBS_PROFILE = 8,   // FP64 per-column u_z power sums per z-chunk
    OBS_ENERGY = 16,   // FP64 1/2 rho u_z^2 partials per tile
};

struct ObserveArgs {
    int flags;
    float *rho;         // [B][nz][ny][nx]
    float *u;           // [B][3][nz][ny][nx]
    float *pops;        // [B][27][nz][ny][nx]
    double *diag_part;  // [tiles][5]
    double *prof_part;  // [B][nzc][P][5]
    double *energy_part;// [tiles]
};

// ring of the coherent-structure sampling: the distinct nodes (columns) it
// touches, and per ring point the indices of its four nodes in that list and
// their bilinear weights
struct RingArgs {
    const int *nodes;   // [n_nodes] columns
    const int *idx;     // [ntheta][4] into nodes
    const double *w;    // [ntheta][4]
    int n_nodes, ntheta;
};

// launchers (return the hipError_t of the launch)
hipError_t launch_step(int storage, const Geom &g, const Tiles &t, const void *src, void *dst, int step_off,
                       hipStream_t s);
// the same for the comparison schemes (g.kind != 0; two-buffer pattern, FP32
// or FP64 storage)
hipError_t launch_step_kind(int storage, const Geom &g, const Tiles &t, const void *src, void *dst, int step_off,
                            hipStream_t s);
// steps n and n+1 in one launch (two-buffer pattern, bounce-back wall, FP32
// or FP16 storage): src holds the state of step n, dst receives step n+2
hipError_t launch_step2(int storage, const Geom &g, const Tiles2 &t, const void *src, void *dst, int step_off,
                        hipStream_t s);
// AA pattern, in place: odd = 0 reads FORM_N and leaves FORM_W, odd = 1 the reverse
hipError_t launch_step_aa(int storage, const Geom &g, const Tiles &t, void *buf, int odd, int step_off, hipStream_t s);
// persistent launch: blocks = groups * per_group workgroups, group q owning
// pipes [q * pipes_per_group, ...); bar: 32 words (error flag) + 32 per
// group.  aa: in place in b0, par = parity of the first step.  cooperative:
// hipLaunchCooperativeKernel; 0: a plain launch (for graph capture).
hipError_t launch_step_persistent(int storage, int aa, const Geom &g, const Tiles &t, void *b0, void *b1, int par,
                                  int nsteps, unsigned *bar, int blocks, int per_group, int pipes_per_group,
                                  int cooperative, hipStream_t s);
int persistent_blocks_per_cu(int storage, int aa, int wall, int block);
hipError_t launch_stream_copy(int storage, const Geom &g, const Tiles &t, const void *src, void *dst, hipStream_t s);
hipError_t launch_observe(int storage, int form, const Geom &g, const Tiles &t, const void *state, const ObserveArgs &o,
                          int step_off, hipStream_t s);
hipError_t launch_init(int storage, int form, const Geom &g, const double *u0, void *state, hipStream_t s);
hipError_t launch_set_pops(int storage, int form, const Geom &g, const float *pops, void *state, hipStream_t s);
hipError_t launch_ring(int storage, int form, const Geom &g, const RingArgs &r, const void *state, float *ring,
                       hipStream_t s);
hipError_t launch_ring_spectrum(const float *ring, int planes, int n, int mmax, const double *tw, double *spec,
                                hipStream_t s);
hipError_t launch_spectrum_mean(const double *spec, int B, int nz, int mmax, double *mean, int *dominant,
                                hipStream_t s);
hipError_t launch_reduce_diag(const Geom &g, const Tiles &t, const double *part, double *out, hipStream_t s);
hipError_t launch_reduce_energy(const Geom &g, const Tiles &t, const double *part, double *out, hipStream_t s);
hipError_t launch_accumulate_energy(const Geom &g, const Tiles &t, const double *part, double scale, double *acc,
                                    hipStream_t s);
hipError_t launch_reduce_profile(const Geom &g, const Tiles &t, const double *part, double *acc, hipStream_t s);
hipError_t launch_fill(void *p, size_t bytes, hipStream_t s);
hipError_t launch_set_step(long long *step_dev, long long value, int add, hipStream_t s);
hipError_t launch_copy(void *dst, const void *src, size_t bytes, hipStream_t s);
// device address, on the current device, of the scratch array of the
// context-free spectrum entry point (looked up once per device)
hipError_t static_scratch(double **out);

// adjoint
struct AdjointArgs {
    const void *state;     // saved forward state holding S^T f^c (or:)
    const void *rec;       // the moments (rho - 1, j) of f^c recorded by the recording step
    const void *lam_in;    // lambda^{c+1} (stored plainly: lambda_i at its own node), float or double
    void *lam_out;         // lambda^c
    double *grad_part;     // [B][nzc][P][3]: FP64 per-column force sensitivities times sigma, summed over the steps
    long long cursor;      // c
    int in_window;         // c in [obs_begin, obs_end)
    int has_next;          // c + 1 was collided (lambda^{c+1} nonzero)
    double energy_weight;  // 1 / (W N_f)
};
hipError_t launch_adjoint(int storage, int precision, const Geom &g, const Tiles &t, const AdjointArgs &a,
                          hipStream_t s);
// one two-buffer step src -> dst that also records the moments of the state
// it consumes into rec ([B][4][population stride] of the arithmetic type)
hipError_t launch_step_record(int storage, const Geom &g, const Tiles &t, const void *src, void *dst, int step_off,
                              void *rec, hipStream_t s);
// acc[b][k] = the column sums over the z-chunks of the gradient partials
hipError_t launch_grad_accumulate(const Geom &g, const Tiles &t, const double *grad_part, double *acc, hipStream_t s);
// grad[b][q] = base[b][q] + sum_k acc[b][k] . shape_q(k)
hipError_t launch_project_grad(const Geom &g, const double *acc, const double *modes, int nq, const double *base,
                               double *grad, hipStream_t s);

}  // namespace lbm
