/*
 * lbm.h -- C-ABI of the MI355X (gfx950) D3Q27 MRT pipe-flow stepper.
 *
 * The method is the lattice Boltzmann scheme of Magacho, Moriconi &
 * Loureiro, "Persistence of large scale coherent structures in a turbulent
 * pipe flow through an improved lattice Boltzmann approach"
 * (arXiv:2405.12082): collide (Eqs. (collision), (mrt), (m*), (Rmrti),
 * (k*f*) of the appendix: multiple-relaxation-time collision in the raw
 * moment basis of Eq. (Mmatrix), relaxation matrix Eq. (lambda), sixth-order
 * Hermite equilibrium Eq. (BoltzmannEquilibriumDistribution), Guo forcing)
 * then stream (Eq. (streaming)), on a D3Q27 lattice inside a circular pipe
 * on a Cartesian mask, axially periodic, driven by a constant body force
 * plus the divergence-free trigger force of Eq. (TurbForce) (Section II.B).
 *
 * Conventions shared by every entry point
 *  - Return value: 0 (LBM_OK) on success, a negative LBM_E* code on error.
 *    Nothing throws across this boundary.  After an error on a context,
 *    lbm_last_error() returns a message.  HIP errors are sticky: once a
 *    call returned LBM_EHIP, every later call on that context does too.
 *  - Memory: the library never allocates device memory.  The caller passes
 *    one device workspace (size from lbm_workspace_bytes) and device output
 *    buffers, and keeps them alive while the context lives.  Host arrays
 *    passed in are copied before the call returns.
 *  - Streams: every device operation is enqueued on the stream given to
 *    lbm_init (a hipStream_t passed as void*).  Calls return once the work
 *    is enqueued, except lbm_init and the calls that return host data
 *    (lbm_diagnostics, lbm_profile_read), which synchronise that stream.
 *  - Threading: one context per stream; calls on one context must not
 *    overlap.
 *  - Geometry: node (x, y, z), 0 <= x < nx etc.; the pipe axis is at
 *    ((nx-1)/2, (ny-1)/2) and a node is fluid iff its distance to the axis
 *    is < radius (radius <= 0: every node is fluid, a fully periodic box).
 *    All axes wrap periodically.  Dense arrays exchanged with the caller
 *    use x fastest: [b][z][y][x]; solid nodes read and write as 0.
 *  - Populations: the library stores deviations g_i = f_i - w_i from the
 *    lattice weights (Eq. (omegas)), in FP32, FP16 (relative to a
 *    per-column reference) or FP64 (storage field).
 *  - Velocity set order: 0 rest; 1-6 (+x,-x,+y,-y,+z,-z); 7-10 xy edges
 *    (++,-+,+-,--); 11-14 xz edges; 15-18 yz edges; 19-26 corners, as in
 *    the appendix.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    LBM_OK = 0,
    LBM_EINVAL = -1, /* invalid argument or configuration */
    LBM_ENOMEM = -2, /* workspace too small */
    LBM_EHIP = -3,   /* HIP runtime error (sticky) */
    LBM_ESTATE = -4, /* call not valid in the current state */
    LBM_ENAN = -5    /* non-finite populations detected */
};

typedef struct lbm_ctx lbm_ctx; /* opaque, owned by the library */

typedef struct {
    int32_t nx, ny, nz;   /* per-pipe box, each >= 1 */
    int32_t batch;        /* independent pipes of the same geometry, >= 1 */
    double radius;        /* pipe radius in lattice units (<= 0: no wall) */
    double tau;           /* relaxation time; omega = 1/tau on moments 4..8 (Eq. (lambda)), > 0.5 */
    double accel_z;       /* constant body acceleration h along z (Section II.B: force density rho h) */
    int32_t n_modes;      /* trigger-force modes m = 1..n_modes (0..6), each cos and sin */
    double kz;            /* streamwise wavenumber k_z of Eq. (TurbForce) */
    double kappa;         /* radial/azimuthal split kappa of Eq. (TurbForce) */
    double l0_frac;       /* l_0 / R: force active for R - l0 - l <= r <= R - l0 */
    double l_frac;        /* l / R */
    double period;        /* forcing period T in steps: time factor sin(2 pi n / T) */
    int64_t force_off_step; /* trigger force applied for steps n < force_off_step */
    int32_t storage;      /* 0: FP32 deviations, FP32 collision; 1: FP16 deviations, FP32
                             collision: a value g_i produced by the node of column y is
                             stored as h = fp16_rne(2^k g_i - E_c(y)) (one rounding of the
                             exact difference) and read as fp32(h / 2^k + E_c(y) / 2^k)
                             (one rounding), with 2^k ~ 1/w_i (4, 16, 64, 256 for
                             |c_i|^2 = 0, 1, 2, 3) and the column's reference E_c(y) =
                             fp32(32/27 d_c(u0(y))), c = c_z of population i, d_c the
                             per-axis factor of the equilibrium (d_0 = -3u^2/2, d_+-1 = +-3u
                             + 3u^2) at the initial streamwise velocity u0 of the column
                             (0 for a rest start): E_c / 2^k is the initial equilibrium
                             deviation, so FP16 holds the departure from it; saved FP16
                             states are relative to their configuration's references;
                             2: FP64 deviations and collision (reference precision, for
                             verification) */
    int32_t wall;         /* 0: halfway bounce-back (the Delta = 1/2 case of Eq. (fbc1));
                             1: interpolated wall of Eqs. (fbc1)/(fbc2) with the exact
                             fraction Delta of each cut link at r = R (two-buffer
                             pattern) */
    int32_t pattern;      /* 0: two buffers (A/B); 1: AA, one buffer updated in place (even
                             steps read and write a node's own slots, odd steps its
                             neighbours'); same results, half the state memory; no
                             adjoint (adjoint must be 0) */
    int32_t init;         /* 0: rest (g = 0); 1: log-law mean profile, f = f^eq(1, u_z(r)) */
    double u_tau;         /* friction velocity u* of the log-law profile (init = 1) */
    int32_t adjoint;      /* adjoint buffers in the workspace: 0 none, 1 FP32 adjoint state,
                             2 FP64 adjoint state (FP64 arithmetic in both) */
    int32_t block;        /* threads per block: 64, 128, 256, 512 (0 = default: 512 for FP32,
                             256 for FP16 and FP64; with wall = 1, 256 for FP32 and FP64, 64
                             for FP16) */
    int32_t zchunk;       /* z planes per thread: 1..64 (0 = default: 1 for FP32, 8 for FP16,
                             2 for FP64; with wall = 1, 2 for FP32 and FP64, 16 for FP16) */
    int32_t xcd_remap;    /* workgroup -> tile order (workgroups go round-robin to the 8 XCDs):
                             0 dispatch order; 1 XCD x takes the x-th eighth of the tiles;
                             G in 2..4096: XCD x takes every eighth chunk of G consecutive
                             tiles (neighbouring tiles share one XCD's L2) */
    int32_t collision;    /* 0: the paper's multiple-relaxation-time collision (Eqs. (mrt),
                             (lambda), (m*)); 1: the single-relaxation-time BGK operator of
                             Eq. (srt), every population relaxed at omega = 1/tau, with
                             f*_i = f_i - omega (f_i - f^eq_i) + (1 - omega/2) F_i
                             (a comparison scheme) */
    int32_t equilibrium;  /* 0: the sixth-order Hermite equilibrium of Eq.
                             (BoltzmannEquilibriumDistribution); 1: the second-order one,
                             f^eq_i = w_i rho (1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u), of the
                             LBM-O(2) scheme compared with in Section III (Table I).  Forcing
                             is F_i = a . grad_u f^eq_i with the chosen equilibrium.  Any
                             choice other than (0, 0) needs FP32 or FP64 storage, the
                             two-buffer pattern and no adjoint; it runs through lbm_step,
                             lbm_step_graph and lbm_recompute (not the persistent or
                             two-step launches) */
} lbm_config;

/* Layout facts of a configuration (host only, no GPU needed). */
typedef struct {
    int64_t n_fluid_columns; /* fluid (x, y) columns of one cross-section */
    int64_t plane_pitch;     /* stored elements per (pipe, population, z) plane */
    int64_t n_fluid_nodes;   /* fluid nodes of one pipe */
    int64_t state_bytes;     /* bytes of one population state (all pipes) */
    int64_t workspace_bytes; /* bytes lbm_init needs */
    int64_t bytes_per_update;/* algorithmic HBM bytes per fluid-node update of lbm_step */
    int64_t population_stride; /* elements between the populations of one pipe: nz * plane_pitch,
                                  padded by 2368 when that is a multiple of 4096 */
    int64_t record_bytes;    /* bytes of one moment record of lbm_recompute_moments (all pipes):
                                [batch][4][population_stride] FP32 (FP64 for FP64 storage),
                                rounded up to 256 */
} lbm_layout;

/* Check a configuration and report its layout.  Host only.
 * Errors: LBM_EINVAL for an invalid configuration (cfg NULL, sizes < 1,
 * tau <= 0.5, n_modes outside 0..6, period <= 0 with n_modes > 0, a
 * cross-section with no fluid column, radius > (min(nx,ny)-1)/2, unknown
 * storage/wall/pattern/init/collision/equilibrium values, block/zchunk out
 * of range, a comparison scheme with FP16 storage, the AA pattern or an
 * adjoint, a pipe one of whose populations would take 4 GiB or more: the
 * population stride (about nz x the fluid columns) times 4 B (FP32), 2 B
 * (FP16) or 8 B (FP64); in FP32 about 1.07 G fluid nodes, 116 GB per state
 * buffer: the kernels use 64-bit pipe and population bases and 32-bit byte
 * offsets within a population), and with an adjoint the same limit on one
 * population of the adjoint state (4 B for adjoint = 1, 8 B for 2). */
int lbm_describe(const lbm_config *cfg, lbm_layout *out);

/* Device workspace size lbm_init needs for cfg.  Host only. */
int lbm_workspace_bytes(const lbm_config *cfg, size_t *bytes);

/* Create a context: validates cfg, builds the z-invariant column tables
 * (fluid-column list, neighbour table, trigger-force shapes from
 * Eq. (TurbForce) with the per-pipe amplitudes) on the host, copies them
 * into the workspace and writes the initial state (step 0).
 *  amps:      host [batch][2*n_modes] doubles, mode m = p/2 + 1 with phase
 *             0 (even p, cos) or pi/(2m) (odd p, sin); amplitude of the
 *             acceleration (replaces h*A_0).  May be NULL if n_modes == 0.
 *  workspace: device memory of at least lbm_workspace_bytes, 256-byte aligned.
 *  stream:    hipStream_t (NULL: the default stream).
 * Synchronises the stream.  *out is NULL on error. */
int lbm_init(const lbm_config *cfg, const double *amps, void *workspace, size_t bytes,
             void *stream, lbm_ctx **out);

/* Enqueue n >= 0 time steps (collide then stream, Eqs. (collision) and
 * (streaming)), one fused stream-collide kernel per step.  Async. */
int lbm_step(lbm_ctx *ctx, int32_t n);

/* Enqueue n steps by replaying a captured HIP graph of k steps (k even,
 * 2 <= k <= 1024; captured on first use and on a change of k) plus eager
 * launches for the remainder.  Async.  Same results as lbm_step. */
int lbm_step_graph(lbm_ctx *ctx, int32_t n, int32_t k);

/* Run n steps as ONE persistent cooperative launch (the paper's collision
 * only: LBM_EINVAL for a comparison scheme): the co-resident
 * workgroups are split into groups that each own whole pipes; a group's
 * workgroups stride over its pipes' tiles and meet at a group barrier before
 * the next step (pipes are independent, so groups never wait for each
 * other).  Same results as lbm_step (bitwise).  The barrier's wait is
 * bounded; if it ever times out the call returns LBM_ESTATE and the state is
 * invalid.  Synchronises the stream. */
int lbm_step_persistent(lbm_ctx *ctx, int32_t n);

/* n steps as replays of a HIP graph holding ONE persistent launch of k steps
 * (the launch of lbm_step_persistent, with the reset of its group counters
 * and the step counter update), k even (2..2^20); one graph per starting
 * buffer is captured on first use and kept until the launch geometry
 * changes.  n mod k remaining steps run as lbm_step_persistent.  Same
 * results as lbm_step (bitwise).  The barrier timeout flag is cleared once
 * before the replays and read once after them: LBM_ESTATE if any barrier
 * timed out (the state is then invalid).  Synchronises the stream.
 * Errors: LBM_EINVAL for n < 0 or a bad k, LBM_EHIP if capture fails. */
int lbm_step_persistent_graph(lbm_ctx *ctx, int32_t n, int32_t k);

/* Change the launch geometry of lbm_step and lbm_step_graph on a live
 * context: threads per block (64, 128, 256, 512), z planes per thread (1..64),
 * tile order (xcd_remap 0..4096, as in lbm_config), pipes per launch (1..batch) and step order
 * (pipe_major 0: every step covers all pipes; 1: within one call, each group
 * of pipes_per_launch pipes runs all n steps before the next group, so a
 * small pipe's working set stays in the 256 MB Infinity Cache).  A value of
 * 0 (-1 for xcd_remap and pipe_major) keeps the current setting.  Drops
 * captured graphs.  Results do not depend on the geometry (the pipes are
 * independent and every node's update is the same arithmetic).
 * Errors: LBM_EINVAL for values out of range. */
int lbm_set_launch(lbm_ctx *ctx, int32_t block, int32_t zchunk, int32_t xcd_remap, int32_t pipes_per_launch,
                   int32_t pipe_major);

/* Run pairs of steps of lbm_step and lbm_step_graph as one launch each
 * (temporal blocking; steps_per_launch = 2) or one step per launch (1).  The
 * two-step kernel cuts the cross-section into 14 x 14 column tiles; a
 * workgroup runs step n on its tile and a ring of halo columns, keeps those
 * post-collision values in LDS, and runs step n+1 on the tile from them one
 * plane behind as it marches along z (zchunk output planes per workgroup,
 * 1..1024), so the state crosses HBM once per two steps.  Each step is the
 * arithmetic of Eqs. (collision), (streaming) and (fbc1) at Delta = 1/2,
 * the same as one step per launch (FP16 storage rounds the intermediate
 * state through its codec).  xcd_remap orders the two-step launch's
 * workgroups as in lbm_config.  Needs the two-buffer pattern, the halfway
 * bounce-back wall and FP32 or FP16 storage.  An odd step count ends with
 * one single step.  0 (-1 for xcd_remap) keeps a setting.  Drops captured
 * graphs.  Errors: LBM_EINVAL for values out of range or an unsupported
 * configuration. */
int lbm_set_fused(lbm_ctx *ctx, int32_t steps_per_launch, int32_t zchunk, int32_t xcd_remap);

/* Current step index n (the state held is f^n, before its collision). */
int lbm_get_step(const lbm_ctx *ctx, int64_t *step);

/* Density and velocity of the current state f^n, Eqs. (macroscopic_rho) and
 * (macroscopic_u), with u = j/rho + a(x, n)/2 (a: the body acceleration of
 * step n).  Device outputs: rho [batch][nz][ny][nx], u [batch][3][nz][ny][nx]
 * (FP32).  Either pointer may be NULL.  Async. */
int lbm_moments(lbm_ctx *ctx, float *rho, float *u);

/* Deviations g_i = f_i - w_i of the current state f^n.  Device output
 * [batch][27][nz][ny][nx] FP32.  Async. */
int lbm_populations(lbm_ctx *ctx, float *g);

/* Replace the state by the given deviations (device [batch][27][nz][ny][nx]
 * FP32; solid entries ignored) and set the step index.  Async. */
int lbm_set_populations(lbm_ctx *ctx, const float *g, int64_t step);

/* FP64 sums of the current state per pipe: host [batch][5] =
 * {sum rho, sum j_x, sum j_y, sum j_z, number of non-finite populations}
 * over fluid nodes, j = sum_i c_i f_i.  Two-pass fixed-order reduction
 * (bitwise reproducible).  Synchronises.  Returns LBM_ENAN (after filling
 * the output) when any population is non-finite. */
int lbm_diagnostics(lbm_ctx *ctx, double *host_out);

/* Failure watchdog of lbm_diagnostics (a guard for long runs): with
 * mass_rel_tol > 0, lbm_diagnostics also returns LBM_ENAN (after filling its
 * output, with a message naming the pipe) when a pipe's mass differs from
 * its reference mass by more than mass_rel_tol relative.  The reference is
 * the mass at the first lbm_diagnostics call after this call, lbm_init,
 * lbm_load or lbm_set_populations.  The halfway bounce-back conserves mass to
 * rounding; the interpolated wall does not (its drift is a property of the
 * scheme).  0 turns the check off (the default).  Host only.
 * Errors: LBM_EINVAL for a negative or non-finite limit. */
int lbm_set_watchdog(lbm_ctx *ctx, double mass_rel_tol);

/* Bounds checks of a checked build (liblbm_checked.so, built from the same
 * sources with LBM_CHECKED=1): the step, observer, ring and adjoint kernels
 * test every population load and store of their gather and store paths
 * against the extent of its population, and every neighbour-table entry and
 * column index against the table; a violation sets a bit and skips the
 * access.  *flags receives the bits recorded since lbm_init (1: neighbour
 * entry out of range, 2: load, 4: store, 8: column or node index); *checked
 * (may be NULL) 1 for a checked build, 0 for the release build, whose flags
 * are always 0.  Synchronises the stream.
 * Errors: LBM_EINVAL for a NULL flags pointer; LBM_EHIP. */
int lbm_check_flags(lbm_ctx *ctx, uint32_t *flags, int32_t *checked);

/* Add the current state's streamwise-velocity power sums to the per-column
 * FP64 accumulators: sum over z of u_z, u_z^2, u_z^3, u_z^4 and the count
 * (statistics of Eq. (urmsformula), pooled over z).  Async. */
int lbm_profile_accumulate(lbm_ctx *ctx);
/* Zero the accumulators.  Async. */
int lbm_profile_reset(lbm_ctx *ctx);
/* Copy the accumulators to host [batch][ny][nx][5] (solid columns 0).
 * Synchronises. */
int lbm_profile_read(lbm_ctx *ctx, double *host_out);

/* Bytes of one saved state (populations, all pipes). */
int lbm_state_bytes(const lbm_ctx *ctx, size_t *bytes);
/* Copy the state to / from caller device memory of lbm_state_bytes bytes;
 * lbm_load also sets the step index.  Async, stream-ordered.  With the AA
 * pattern the buffer's layout depends on the parity of the step, so a saved
 * state must be loaded at a step of the same parity. */
int lbm_save(lbm_ctx *ctx, void *dst, int64_t *step);
int lbm_load(lbm_ctx *ctx, const void *src, int64_t step);

/* Discrete adjoint of lbm_step (requires cfg.adjoint = 1 or 2).
 * Forward map of one step: f^{n+1} = S C(f^n, a^n), C the collision at every
 * fluid node, S the streaming with the wall.  Objective:
 *     J = 1/W sum_{n in [obs_begin, obs_end)} E(f^n),
 *     E(f^n) = (1/N_f) sum_x 1/2 rho u_z^2 with u_z = j_z/rho + a_z(x, n)/2,
 * the time-averaged streamwise kinetic energy, W = obs_end - obs_begin.
 * The adjoint state lambda^n = dJ/df^n lives in the workspace (FP32 or FP64;
 * the vector-Jacobian products are computed in FP64 in either case):
 *     lambda^c = (dC/df^c)^T S^T lambda^{c+1} + dE_c/df^c [c in window],
 * with lambda^{N+1} = 0 for the last state N = obs_end - 1.
 *
 * lbm_adjoint_reset: lambda := 0, stores the window and sets the cursor c
 * to obs_end - 1.  Async.
 * lbm_adjoint_step: n >= 1 reverse steps.  fwd_states points to n saved
 * states (lbm_save layout, device memory) f^{c-n+1} .. f^c in forward order,
 * state_stride bytes apart; they are consumed last to first, each one
 * producing lambda^c and moving the cursor to c - 1.  The gradient
 *     dJ/d amps[b][q] = sum_c sum_x [(dC/da)^T S^T lambda^{c+1} + dE_c/da] . da(x,c)/d amps[b][q]
 * is accumulated in FP64 per column over the steps of the sweep (fixed
 * order), and each call writes grad = (the values grad held at the sweep's
 * first call) + the gradient of all steps consumed so far (device
 * [batch][2*n_modes] doubles, caller-owned; not modified by the caller
 * between the calls of one sweep), so the result does not depend on how the
 * sweep is split into calls.  Once f^0 is consumed the gradient is complete.
 * Errors: LBM_ESTATE if the adjoint buffers are absent, no reset was made,
 * or the cursor would move below 0.  Async. */
int lbm_adjoint_reset(lbm_ctx *ctx, int64_t obs_begin, int64_t obs_end);
int lbm_adjoint_step(lbm_ctx *ctx, int32_t n, const void *fwd_states, size_t state_stride,
                     double *grad);
/* Objective E(f^n) of the current forward state per pipe, FP64, host
 * [batch].  Synchronises. */
int lbm_energy(lbm_ctx *ctx, double *host_out);
/* Same value added to a device accumulator: acc[b] += E_b(f^n) (device
 * [batch] doubles, caller-owned), fixed-order FP64 reduction.  Async. */
int lbm_energy_accumulate(lbm_ctx *ctx, double *acc);

/* Record forward states for checkpoint-and-recompute without touching the
 * context's own state: ring[0] := start (a saved state, lbm_save layout, of
 * step s0; no copy when start == ring), then ring[j+1] := one step of
 * ring[j] at step index s0 + j, for j = 0 .. n-2.  ring: device memory for
 * n states, stride bytes apart (stride >= lbm_state_bytes, multiple of 256).
 * The states are exactly those lbm_step would produce.  Two-buffer pattern
 * only (LBM_EINVAL otherwise).  Async. */
int lbm_recompute(lbm_ctx *ctx, const void *start, int64_t s0, int32_t n, void *ring, size_t stride);

/* Checkpoint-and-recompute with moment records: the collision depends on the
 * state only through rho, j and the stress moments m_4..m_8 (appendix,
 * Eqs. (m*)-(k*f*)), and its Jacobian only through rho and u, so the reverse
 * step needs of each forward state f^c only rho - 1 and j = sum c_i f_i:
 * 16 B per node (32 B in FP64) instead of the state's 108 B (216 B).
 * lbm_recompute_moments: scratch[0] := start (a saved state of step s0; no
 * copy when start == scratch), then n steps of the two-buffer pattern
 * alternating between the two scratch states (device memory, stride bytes
 * apart: stride >= lbm_state_bytes, multiple of 256), step j (state of step
 * s0 + j) recording the moments of the state it consumes into records[j]
 * (device memory, record_stride bytes apart: record_stride >=
 * lbm_layout.record_bytes, multiple of 256; layout [batch][q][z P + k], q =
 * rho - 1, j_x, j_y, j_z, each q a region of population_stride elements; in
 * the collision's arithmetic type).  The states are exactly those lbm_step
 * would produce; the context's own state is untouched.  start is scratch
 * state 0 or outside both scratch states.  Two-buffer pattern and the
 * paper's scheme only (LBM_EINVAL otherwise).  Async.
 * lbm_adjoint_step_moments: lbm_adjoint_step with n records of
 * lbm_recompute_moments (moments of f^{c-n+1} .. f^c in forward order,
 * record_stride bytes apart) in place of the saved states; the same
 * arithmetic from the recorded moments (the forward collision's own, in its
 * arithmetic type) instead of FP64 sums of the gathered state.  Errors and
 * cursor as lbm_adjoint_step.  Async. */
int lbm_recompute_moments(lbm_ctx *ctx, const void *start, int64_t s0, int32_t n, void *scratch, size_t stride,
                          void *records, size_t record_stride);
int lbm_adjoint_step_moments(lbm_ctx *ctx, int32_t n, const void *records, size_t record_stride, double *grad);

/* n steps of the context's own state, as lbm_step does them, step j
 * recording the moments of the state it consumes (the state of step
 * c + j, c the step index before the call) into records[j] (layout and
 * stride as lbm_recompute_moments).  With the records of every step of a
 * forward run kept in device memory (record_bytes each: 39 MB for a
 * 96x96x384 pipe, 78 GB for 2000 steps of it) the reverse sweep
 * (lbm_adjoint_step_moments over them) needs no recompute.  Two-buffer
 * pattern, one step per launch and the paper's scheme only (LBM_EINVAL
 * otherwise).  Async. */
int lbm_step_recording(lbm_ctx *ctx, int32_t n, void *records, size_t record_stride);

/* Measurement aid: enqueue n copies of the current state buffer into the
 * other buffer with the launch geometry of lbm_step (27 aligned loads and 27
 * non-temporal stores per fluid node, no arithmetic): the HBM rate of the
 * step's access pattern alone, a reference point for the step (which can
 * run faster: the step kernel's loads and arithmetic overlap differently).
 * Leaves the state
 * unchanged (the copy goes to the spare buffer; with the AA pattern the
 * buffer is copied onto itself).  Async. */
int lbm_stream_copy(lbm_ctx *ctx, int32_t n);

/* Coherent-structure identification, Section II.C.
 *
 * lbm_ring_sample: the streamwise velocity u_z (as lbm_moments reports it,
 * at the current step) on the circle r = r0 (lattice units; the paper uses
 * r0 = 0.78 R) at ntheta points theta_j = 2 pi j / ntheta, theta =
 * atan2(y - y_c, x - x_c), by bilinear interpolation of the four
 * surrounding nodes, for every plane z of every pipe.  ring: device
 * [batch][nz][ntheta] float.  Async (the first call for a new (r0, ntheta)
 * synchronises the stream once).  LBM_EINVAL for ntheta outside 4..4096,
 * r0 <= 0, or a ring that touches a solid node.
 *
 * lbm_ring_spectrum: for each plane the Fourier transform of the azimuthal
 * correlation R_uu(dtheta) = <du(theta0) du(theta0 + dtheta)>_theta0 / u_rms^2
 * of the ring samples (du about the plane's ring mean), which equals the
 * normalised power |U(m)|^2 / sum_j du_j^2 of the DFT U of du, for modes
 * m = 0..mmax (m = 0 is 0): spec, device [batch][nz][mmax+1] double.
 * mean (device [batch][mmax+1] double, may be NULL): the plane average;
 * dominant (device [batch] int32, may be NULL; needs mean): the dominant
 * azimuthal mode, the highest peak of the power of the averaged transform
 * among m >= 1 (0 if it vanishes).  ring: as written by lbm_ring_sample
 * (ntheta per plane).  Async.  LBM_EINVAL for NULL ring/spec, ntheta
 * outside 4..4096, mmax outside 1..ntheta/2, dominant without mean. */
int lbm_ring_sample(lbm_ctx *ctx, double r0, int32_t ntheta, float *ring);
int lbm_ring_spectrum(lbm_ctx *ctx, const float *ring, int32_t ntheta, int32_t mmax, double *spec, double *mean,
                      int32_t *dominant);

/* lbm_ring_spectrum without a context, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses
 * that forbid hipMalloc): the same transform and plane average of ring
 * samples of batch pipes of nz planes (ring: device [batch][nz][ntheta]
 * float; spec, mean, dominant as in lbm_ring_spectrum), enqueued on stream
 * (a hipStream_t, NULL: the default stream).  It allocates nothing: its
 * only scratch, the twiddle table, is a library-owned device array of 4096
 * points (64 KiB) per GPU, held until the process ends, whose address the
 * library looks up once per device (at lbm_init, or at the first call on
 * that device, which should then be made outside graph capture).  Every
 * call rewrites the part of the table it uses; calls that overlap on one
 * GPU share the table and race.  Twiddles are computed on the device, so
 * results equal lbm_ring_spectrum's to FP64 rounding (the dominant mode
 * exactly, barring ties within rounding).  Async.
 * Errors: LBM_EINVAL for NULL ring/spec, batch or nz < 1, batch * nz >
 * 2^31 - 1, ntheta outside 4..4096 (the scratch limit), mmax outside
 * 1..ntheta/2, dominant without mean; LBM_EHIP for a HIP error. */
int lbm_ring_spectrum_static(const float *ring, int32_t batch, int32_t nz, int32_t ntheta, int32_t mmax,
                             double *spec, double *mean, int32_t *dominant, void *stream);

/* Message of the last error on ctx ("" if none; a static message if ctx is NULL). */
const char *lbm_last_error(const lbm_ctx *ctx);
/* Release the context (not the caller's memory).  Synchronises its stream. */
void lbm_destroy(lbm_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
