/*
 * lbm_oracle.h -- plain FP64 CPU reference for the D3Q27 MRT pipe-flow
 * stepper of Magacho, Moriconi & Loureiro (arXiv:2405.12082).
 *
 * TEST INFRASTRUCTURE ONLY.  This oracle exists to check the HIP library
 * against the paper.  It shares no code, header or table with the HIP path;
 * only tests, the smoke check and the CPU-baseline leg of the benchmark may
 * load it.  It is written for clarity, not speed: dense 27x27 moment
 * transforms, the printed closed forms for m^eq and R, and per-node loops.
 *
 * Storage: the distribution f is kept as full populations (not deviations),
 * node-major: f[((z*ny + y)*nx + x)*27 + i].  Exported arrays use the layout
 * [i][z][y][x] (populations) and [z][y][x] (scalars).
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t nx, ny, nz;       /* box; pipe axis along z at ((nx-1)/2, (ny-1)/2) */
    double radius;            /* node is fluid iff its distance to the axis is < radius */
    double tau;               /* relaxation time: omega = 1/tau on m_4..m_8, nu = (tau-1/2)/3 */
    double accel_z;           /* constant body acceleration h along z */
    int32_t n_modes;          /* azimuthal modes m = 1..n_modes of the trigger force, cos and sin */
    double kz, kappa, l0_frac, l_frac, period;  /* Eq. (TurbForce) parameters; period T in steps */
    int64_t force_off_step;   /* trigger force active for steps n < force_off_step */
    int32_t wall;             /* 0: halfway bounce-back, 1: Bouzidi, Eqs. (fbc1)-(fbc2) */
    int32_t init;             /* 0: rest (f = w), 1: log-law mean profile (f = f^eq) */
    double u_tau;             /* friction velocity used by the log-law initial profile */
    int32_t collision;        /* 0: MRT of the appendix (Eq. (m*)); 1: SRT/BGK, Eq. (srt) */
    int32_t equilibrium;      /* 0: sixth-order Hermite equilibrium; 1: second-order (LBM-O(2)) */
} orc_config;

typedef struct orc_pipe orc_pipe;

/* --- lattice and per-node formulas (appendix) --- */
void orc_lattice(int32_t c[27 * 3], double w[27], int32_t opp[27]);
void orc_moment_matrix(double A[27 * 27]);      /* A[k*27+i] = M_k(c_i) */
void orc_moment_matrix_inverse(double Ai[27 * 27]);
void orc_feq(double rho, const double u[3], double feq[27]);
void orc_meq(double rho, const double u[3], double meq[27]);
void orc_rmrt(double rho, const double u[3], const double F[3], double R[27]);
void orc_collide(const double f[27], const double a[3], double omega, double fs[27]);
/* second-order equilibrium and its forcing term (comparison scheme), and the
 * collision of a given kind (collision, equilibrium as in orc_config) */
void orc_feq2(double rho, const double u[3], double feq[27]);
void orc_force2(double rho, const double u[3], const double a[3], double F[27]);
void orc_collide_kind(const double f[27], const double a[3], double omega, int32_t collision,
                      int32_t equilibrium, double fs[27]);
/* complex-step variants: arguments are interleaved (re, im) pairs */
void orc_feq_cplx(const double rho[2], const double u[6], double feq[54]);
void orc_meq_cplx(const double rho[2], const double u[6], double meq[54]);
void orc_collide_cplx(const double f[54], const double a[6], double omega, double fs[54]);
/* Bouzidi boundary value, Eqs. (fbc1)-(fbc2): the unknown incoming
 * population from f*_out(x) (population leaving toward the wall), f*_in(x)
 * (own node, incoming direction) and f*_out(x_ff); has_ff = 0 falls back to
 * halfway bounce-back. */
double orc_bouzidi(double delta, double fs_out_x, double fs_in_x, double fs_out_xff, int32_t has_ff);
/* Fraction Delta in (0, 1] of the link from fluid node (x, y) along the
 * in-plane part of direction d at which it meets the wall r = R (ray-circle
 * intersection), as used by the streaming with the Bouzidi wall. */
double orc_wall_fraction(const orc_config *cfg, int32_t x, int32_t y, int32_t d);
/* Trigger force of Eq. (TurbForce) summed over modes, at a point, with the
 * time factor sin(2 pi t / T) taken as 1; Cartesian components. */
void orc_trigger_shape(const orc_config *cfg, const double *amps, double x, double y, double z,
                       double out[3]);

/* Body acceleration a(x, n) = h z^ + sin(2 pi n / T) [n < force_off_step] x
 * trigger shape, at node (x, y, z) and step n. */
void orc_force_at(const orc_config *cfg, const double *amps, int32_t x, int32_t y, int32_t z, int64_t n,
                  double out[3]);

/* --- pipe stepper --- */
orc_pipe *orc_pipe_new(const orc_config *cfg, const double *amps /* [2*n_modes] or NULL */);
void orc_pipe_free(orc_pipe *p);
int64_t orc_pipe_step_index(const orc_pipe *p);
int64_t orc_pipe_fluid_count(const orc_pipe *p);
void orc_pipe_fluid_mask(const orc_pipe *p, uint8_t *mask /* [z][y][x] */);
void orc_pipe_step(orc_pipe *p, int32_t n);
void orc_pipe_stream(orc_pipe *p);                 /* f <- S f (streaming alone) */
void orc_pipe_get_f(const orc_pipe *p, double *f /* [27][z][y][x] */);
void orc_pipe_set_f(orc_pipe *p, const double *f /* [27][z][y][x] */, int64_t step);
void orc_pipe_force(const orc_pipe *p, int64_t n, double *a /* [3][z][y][x] */);
void orc_pipe_moments(const orc_pipe *p, double *rho, double *u /* [3][z][y][x] */);
void orc_pipe_sums(const orc_pipe *p, double out[4]); /* sum rho, sum j (raw first moments) */
double orc_pipe_energy(const orc_pipe *p);           /* (1/N_f) sum 1/2 rho u_z^2 */
int32_t orc_num_threads(void);

/* --- adjoint: gradient of the time-averaged streamwise energy ---
 * J = 1/(end-begin) * sum_{n=begin}^{end-1} E(f^n), E = (1/N_f) sum_x 1/2 rho u_z^2,
 * starting from the configured initial state and stepping end-1 times.
 * grad[p] = dJ/d amps[p].  Returns J. */
double orc_adjoint_gradient(const orc_config *cfg, const double *amps, int64_t obs_begin,
                            int64_t obs_end, double *grad);
/* Same gradient by the complex-step tangent of the whole run (one complex
 * forward run per amplitude).  Returns J. */
double orc_tangent_gradient(const orc_config *cfg, const double *amps, int64_t obs_begin,
                            int64_t obs_end, double *grad);
/* J alone (plain FP64 forward run). */
double orc_objective(const orc_config *cfg, const double *amps, int64_t obs_begin, int64_t obs_end);

#ifdef __cplusplus
}
#endif
#endif
