/*
 * lbm_oracle.c -- plain FP64 CPU reference for the D3Q27 MRT pipe-flow
 * stepper of Magacho, Moriconi & Loureiro (arXiv:2405.12082).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark to check the HIP library against the
 * paper.  It shares no code with the HIP path.  Every step is the paper's
 * definition written out, in the paper's order:
 *   collide (Eqs. (collision), (mrt), (m*), (Rmrti), (k*f*), appendix)
 *   then stream (Eq. (streaming)) with the pipe wall (Eqs. (fbc1)-(fbc2)).
 *
 * Readings of points the paper leaves open (each one is listed, with its
 * reason, in the design notes of the repository):
 *  - the velocity row c_x printed in the appendix has 27 entries once its
 *    missing comma is restored; opposites are found by search;
 *  - one moment matrix A with A[k][i] = M_k(c_i): m = A f, f* = A^{-1} m*;
 *  - F in Eqs. (m*)/(Rmrti) is the body acceleration a, u = j/rho + a/2,
 *    and the same shifted u enters m^eq and R;
 *  - tensor Hermite polynomials with every index used at most twice factor
 *    into 1-D factors h_0 = 1, h_1 = c, h_2 = c^2 - c_s^2;
 *  - pipe axis at ((nx-1)/2, (ny-1)/2), fluid iff r < R; periodic wrap on
 *    every axis (radius <= 0 means no wall: a fully periodic box);
 *  - trigger force: mode (m, phase) is Eq. (TurbForce) with k_theta = m and
 *    theta -> theta - phase, phase in {0, pi/(2m)}, amplitude h*A_0 -> amps,
 *    time t = step index n, active for n < force_off_step.
 */
#include "lbm_oracle.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double _Complex cplx;

/* ---------------------------------------------------------------------- */
/* Lattice: D3Q27 velocities as printed in the appendix, weights Eq. (omegas) */
/* ---------------------------------------------------------------------- */
static const int ORC_C[27][3] = {
    /* rest */ {0, 0, 0},
    /* faces */ {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    /* edges */ {1, 1, 0}, {-1, 1, 0}, {1, -1, 0}, {-1, -1, 0},
    {1, 0, 1}, {-1, 0, 1}, {1, 0, -1}, {-1, 0, -1},
    {0, 1, 1}, {0, -1, 1}, {0, 1, -1}, {0, -1, -1},
    /* corners */ {1, 1, 1}, {-1, 1, 1}, {1, -1, 1}, {-1, -1, 1},
    {1, 1, -1}, {-1, 1, -1}, {1, -1, -1}, {-1, -1, -1}};

static double ORC_W[27];
static int ORC_OPP[27];
static double ORC_A[27][27];
static double ORC_AINV[27][27];

/* 1-D Hermite factor of order n (0, 1, 2) with c_s^2 = 1/3 */
static double herm1(int n, double c)
{
    if (n == 0) return 1.0;
    if (n == 1) return c;
    return c * c - 1.0 / 3.0;
}
/* tensor Hermite polynomial with index counts (nx, ny, nz), each <= 2 */
static double herm3(int nx, int ny, int nz, double cx, double cy, double cz)
{
    return herm1(nx, cx) * herm1(ny, cy) * herm1(nz, cz);
}

/* moment basis of Eq. (Mmatrix): M_k evaluated at velocity (x, y, z) */
static double moment_basis(int k, double x, double y, double z)
{
    const double x2 = x * x, y2 = y * y, z2 = z * z;
    switch (k) {
    case 0: return 1.0;
    case 1: return x;
    case 2: return y;
    case 3: return z;
    case 4: return x * y;
    case 5: return x * z;
    case 6: return y * z;
    case 7: return x2 - y2;
    case 8: return x2 - z2;
    case 9: return x2 + y2 + z2;
    case 10: return x * y2 + x * z2;
    case 11: return x2 * y + y * z2;
    case 12: return x2 * z + y2 * z;
    case 13: return x * y2 - x * z2;
    case 14: return x2 * y - y * z2;
    case 15: return x2 * z - y2 * z;
    case 16: return x * y * z;
    case 17: return x2 * y2 + x2 * z2 + y2 * z2;
    case 18: return x2 * y2 + x2 * z2 - y2 * z2;
    case 19: return x2 * y2 - x2 * z2;
    case 20: return x2 * y * z;
    case 21: return x * y2 * z;
    case 22: return x * y * z2;
    case 23: return x * y2 * z2;
    case 24: return x2 * y * z2;
    case 25: return x2 * y2 * z;
    case 26: return x2 * y2 * z2;
    }
    return 0.0;
}

/* Gauss-Jordan inversion with partial pivoting, FP64 */
static int invert27(const double in[27][27], double out[27][27])
{
    double a[27][54];
    for (int r = 0; r < 27; ++r)
        for (int c = 0; c < 54; ++c) a[r][c] = (c < 27) ? in[r][c] : (c - 27 == r ? 1.0 : 0.0);
    for (int col = 0; col < 27; ++col) {
        int piv = col;
        for (int r = col + 1; r < 27; ++r)
            if (fabs(a[r][col]) > fabs(a[piv][col])) piv = r;
        if (a[piv][col] == 0.0) return -1;
        if (piv != col)
            for (int c = 0; c < 54; ++c) {
                double t = a[col][c];
                a[col][c] = a[piv][c];
                a[piv][c] = t;
            }
        const double d = a[col][col];
        for (int c = 0; c < 54; ++c) a[col][c] /= d;
        for (int r = 0; r < 27; ++r) {
            if (r == col || a[r][col] == 0.0) continue;
            const double fct = a[r][col];
            for (int c = 0; c < 54; ++c) a[r][c] -= fct * a[col][c];
        }
    }
    for (int r = 0; r < 27; ++r)
        for (int c = 0; c < 27; ++c) out[r][c] = a[r][c + 27];
    return 0;
}

static int orc_tables_ready = 0;
static void orc_setup(void)
{
    if (orc_tables_ready) return;
    const double w0 = 8.0 / 27.0;
    for (int i = 0; i < 27; ++i) {
        const int s = ORC_C[i][0] * ORC_C[i][0] + ORC_C[i][1] * ORC_C[i][1] + ORC_C[i][2] * ORC_C[i][2];
        ORC_W[i] = (s == 0) ? w0 : (s == 1) ? w0 / 4.0 : (s == 2) ? w0 / 16.0 : w0 / 64.0;
        ORC_OPP[i] = -1;
        for (int j = 0; j < 27; ++j)
            if (ORC_C[j][0] == -ORC_C[i][0] && ORC_C[j][1] == -ORC_C[i][1] && ORC_C[j][2] == -ORC_C[i][2])
                ORC_OPP[i] = j;
    }
    for (int k = 0; k < 27; ++k)
        for (int i = 0; i < 27; ++i) ORC_A[k][i] = moment_basis(k, ORC_C[i][0], ORC_C[i][1], ORC_C[i][2]);
    invert27((const double(*)[27])ORC_A, ORC_AINV);
    orc_tables_ready = 1;
}
__attribute__((constructor)) static void orc_ctor(void) { orc_setup(); }

/* per-node formulas, instantiated for real and complex scalars */
#define SCALAR double
#define FN(name) name##_r
#include "formulas.inc"
#undef SCALAR
#undef FN
#define SCALAR cplx
#define FN(name) name##_c
#include "formulas.inc"
#undef SCALAR
#undef FN

/* ---------------------------------------------------------------------- */
/* exported per-node API                                                   */
/* ---------------------------------------------------------------------- */
void orc_lattice(int32_t c[27 * 3], double w[27], int32_t opp[27])
{
    for (int i = 0; i < 27; ++i) {
        for (int d = 0; d < 3; ++d) c[3 * i + d] = ORC_C[i][d];
        w[i] = ORC_W[i];
        opp[i] = ORC_OPP[i];
    }
}
void orc_moment_matrix(double A[27 * 27]) { memcpy(A, ORC_A, sizeof(ORC_A)); }
void orc_moment_matrix_inverse(double Ai[27 * 27]) { memcpy(Ai, ORC_AINV, sizeof(ORC_AINV)); }
void orc_feq(double rho, const double u[3], double feq[27]) { orc_feq_r(rho, u, feq); }
void orc_meq(double rho, const double u[3], double meq[27]) { orc_meq_r(rho, u, meq); }
void orc_rmrt(double rho, const double u[3], const double F[3], double R[27]) { orc_rmrt_r(rho, u, F, R); }
void orc_collide(const double f[27], const double a[3], double omega, double fs[27])
{
    orc_collide_r(f, a, omega, fs, NULL, NULL);
}
void orc_feq2(double rho, const double u[3], double feq[27]) { orc_feq2_r(rho, u, feq); }
void orc_force2(double rho, const double u[3], const double a[3], double F[27]) { orc_force2_r(rho, u, a, F); }
void orc_collide_kind(const double f[27], const double a[3], double omega, int32_t collision,
                      int32_t equilibrium, double fs[27])
{
    orc_collide_kind_r(f, a, omega, collision, equilibrium, fs, NULL, NULL);
}
static cplx mkc(const double *ri) { return ri[0] + I * ri[1]; }
static void putc2(double *ri, cplx v)
{
    ri[0] = creal(v);
    ri[1] = cimag(v);
}
void orc_feq_cplx(const double rho[2], const double u[6], double feq[54])
{
    cplx uc[3] = {mkc(u), mkc(u + 2), mkc(u + 4)}, out[27];
    orc_feq_c(mkc(rho), uc, out);
    for (int i = 0; i < 27; ++i) putc2(feq + 2 * i, out[i]);
}
void orc_meq_cplx(const double rho[2], const double u[6], double meq[54])
{
    cplx uc[3] = {mkc(u), mkc(u + 2), mkc(u + 4)}, out[27];
    orc_meq_c(mkc(rho), uc, out);
    for (int i = 0; i < 27; ++i) putc2(meq + 2 * i, out[i]);
}
void orc_collide_cplx(const double f[54], const double a[6], double omega, double fs[54])
{
    cplx fc[27], ac[3] = {mkc(a), mkc(a + 2), mkc(a + 4)}, out[27];
    for (int i = 0; i < 27; ++i) fc[i] = mkc(f + 2 * i);
    orc_collide_c(fc, ac, omega, out, NULL, NULL);
    for (int i = 0; i < 27; ++i) putc2(fs + 2 * i, out[i]);
}

/* Bouzidi interpolation, Eqs. (fbc1) (Delta >= 1/2) and (fbc2) (Delta < 1/2) */
double orc_bouzidi(double delta, double fs_out_x, double fs_in_x, double fs_out_xff, int32_t has_ff)
{
    if (delta >= 0.5) return fs_out_x / (2.0 * delta) + (2.0 * delta - 1.0) / (2.0 * delta) * fs_in_x;
    if (!has_ff) return fs_out_x;
    return 2.0 * delta * fs_out_x + (1.0 - 2.0 * delta) * fs_out_xff;
}

/* ---------------------------------------------------------------------- */
/* geometry and forcing                                                    */
/* ---------------------------------------------------------------------- */
static double axis_x(const orc_config *c) { return 0.5 * (c->nx - 1); }
static double axis_y(const orc_config *c) { return 0.5 * (c->ny - 1); }

static int is_fluid_xy(const orc_config *c, int x, int y)
{
    if (c->radius <= 0.0) return 1;
    const double dx = x - axis_x(c), dy = y - axis_y(c);
    return sqrt(dx * dx + dy * dy) < c->radius;
}

/* One mode of Eq. (TurbForce) at unit time factor, in cylindrical
 * components (F_r, F_theta, F_z); zero outside R-l0-l <= r <= R-l0. */
static void turbforce_mode(const orc_config *c, double amp, int ktheta, double phase, double r,
                           double theta, double z, double *Fr, double *Ft, double *Fz)
{
    const double R = c->radius, L = (double)c->nz;
    const double l0 = c->l0_frac * R, l = c->l_frac * R;
    *Fr = *Ft = *Fz = 0.0;
    if (r < R - l0 - l || r > R - l0) return;
    const double th = theta - phase;
    const double arg = 2.0 * M_PI * (R - r - l0) / l;
    const double zc = cos(c->kz * 2.0 * M_PI * z / L), zs = sin(c->kz * 2.0 * M_PI * z / L);
    *Fr = -amp * c->kappa * (R / r) * (c->kz * l / L) * (1.0 - cos(arg)) * zc * cos(ktheta * th);
    *Ft = amp * (1.0 - c->kappa) * (c->kz / ktheta) * (2.0 * M_PI * R / L) * sin(arg) * zc * sin(ktheta * th);
    *Fz = -amp * (R / r) * sin(arg) * zs * cos(ktheta * th);
}

/* Cartesian trigger-force shape for one amplitude index p (mode m = p/2+1,
 * phase 0 for even p (cos), pi/(2m) for odd p (sin)) with amplitude amp */
static void trigger_mode_cart(const orc_config *c, int p, double amp, double x, double y, double z,
                              double out[3])
{
    out[0] = out[1] = out[2] = 0.0;
    if (c->radius <= 0.0) return;
    const double dx = x - axis_x(c), dy = y - axis_y(c);
    const double r = sqrt(dx * dx + dy * dy);
    if (r <= 0.0) return;
    const double theta = atan2(dy, dx);
    const int m = p / 2 + 1;
    const double phase = (p % 2) ? M_PI / (2.0 * m) : 0.0;
    double Fr, Ft, Fz;
    turbforce_mode(c, amp, m, phase, r, theta, z, &Fr, &Ft, &Fz);
    out[0] = Fr * cos(theta) - Ft * sin(theta);
    out[1] = Fr * sin(theta) + Ft * cos(theta);
    out[2] = Fz;
}

void orc_trigger_shape(const orc_config *c, const double *amps, double x, double y, double z, double out[3])
{
    out[0] = out[1] = out[2] = 0.0;
    for (int p = 0; p < 2 * c->n_modes; ++p) {
        double t[3];
        trigger_mode_cart(c, p, amps[p], x, y, z, t);
        for (int d = 0; d < 3; ++d) out[d] += t[d];
    }
}

/* time factor sin(2 pi n / T), switched off from force_off_step on */
static double time_factor(const orc_config *c, int64_t n)
{
    if (c->n_modes <= 0 || n >= c->force_off_step) return 0.0;
    return sin(2.0 * M_PI * (double)n / c->period);
}

/* body acceleration a(x, n) at node (x, y, z), step n: h z^ + time factor x trigger shape */
void orc_force_at(const orc_config *c, const double *amps, int32_t x, int32_t y, int32_t z, int64_t n,
                  double out[3])
{
    double s[3];
    orc_trigger_shape(c, amps, x, y, z, s);
    const double tf = time_factor(c, n);
    out[0] = tf * s[0];
    out[1] = tf * s[1];
    out[2] = c->accel_z + tf * s[2];
}

/* ---------------------------------------------------------------------- */
/* pipe state                                                              */
/* ---------------------------------------------------------------------- */
struct orc_pipe {
    orc_config cfg;
    double amps[12];
    int64_t step;
    size_t nnode;
    int64_t nfluid;
    uint8_t *fluid; /* [z][y][x] */
    double *f;      /* f^n, node-major */
    double *fs;     /* post-collision scratch */
    double *shape;  /* summed trigger shape at unit time factor, [node][3] */
};

static size_t node_index(const orc_config *c, int x, int y, int z)
{
    return ((size_t)z * c->ny + y) * c->nx + x;
}
static int wrap(int v, int n) { return ((v % n) + n) % n; }

/* fractional distance Delta in (0,1] from fluid node (x,y) along the in-plane
 * part of direction d to the wall r = R (ray-circle intersection) */
static double wall_fraction(const orc_config *c, int x, int y, int d)
{
    const double px = x - axis_x(c), py = y - axis_y(c);
    const double vx = ORC_C[d][0], vy = ORC_C[d][1];
    const double aa = vx * vx + vy * vy;
    const double bb = 2.0 * (px * vx + py * vy);
    const double cc = px * px + py * py - c->radius * c->radius;
    return (-bb + sqrt(bb * bb - 4.0 * aa * cc)) / (2.0 * aa);
}

double orc_wall_fraction(const orc_config *c, int32_t x, int32_t y, int32_t d)
{
    return wall_fraction(c, x, y, d);
}

/* Terms of the streaming step, Eq. (streaming), for population i at fluid
 * node (x,y,z): f_i(x, n+1) = sum_t coef[t] * fs_{pop[t]}(src[t], n).
 * Shared by the forward stream and its exact transpose. */
static int stream_terms(const orc_pipe *p, int x, int y, int z, int i, size_t src[2], int pop[2],
                        double coef[2])
{
    const orc_config *c = &p->cfg;
    const int xs = wrap(x - ORC_C[i][0], c->nx), ys = wrap(y - ORC_C[i][1], c->ny);
    const int zs = wrap(z - ORC_C[i][2], c->nz);
    const size_t here = node_index(c, x, y, z), s = node_index(c, xs, ys, zs);
    if (p->fluid[s]) {
        src[0] = s;
        pop[0] = i;
        coef[0] = 1.0;
        return 1;
    }
    const int io = ORC_OPP[i];
    if (c->wall == 0) { /* halfway bounce-back: the Delta = 1/2 case of Eq. (fbc1) */
        src[0] = here;
        pop[0] = io;
        coef[0] = 1.0;
        return 1;
    }
    const double delta = wall_fraction(c, x, y, io);
    if (delta >= 0.5) { /* Eq. (fbc1) */
        src[0] = here;
        pop[0] = io;
        coef[0] = 1.0 / (2.0 * delta);
        src[1] = here;
        pop[1] = i;
        coef[1] = (2.0 * delta - 1.0) / (2.0 * delta);
        return 2;
    }
    /* Eq. (fbc2): x_ff = x + c_i */
    const int xf = wrap(x + ORC_C[i][0], c->nx), yf = wrap(y + ORC_C[i][1], c->ny);
    const int zf = wrap(z + ORC_C[i][2], c->nz);
    const size_t ff = node_index(c, xf, yf, zf);
    if (!p->fluid[ff]) {
        src[0] = here;
        pop[0] = io;
        coef[0] = 1.0;
        return 1;
    }
    src[0] = here;
    pop[0] = io;
    coef[0] = 2.0 * delta;
    src[1] = ff;
    pop[1] = io;
    coef[1] = 1.0 - 2.0 * delta;
    return 2;
}

/* log-law mean profile (Section II.B initial condition), u_z at radius r */
static double loglaw_uz(const orc_config *c, double r)
{
    const double nu = (c->tau - 0.5) / 3.0;
    const double dplus = (c->radius - r) * c->u_tau / nu;
    const double U = (dplus <= 10.8) ? dplus : log(dplus) / 0.4 + 5.0;
    return c->u_tau * U;
}

static void initial_state(orc_pipe *p)
{
    const orc_config *c = &p->cfg;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < c->nz; ++z)
        for (int y = 0; y < c->ny; ++y)
            for (int x = 0; x < c->nx; ++x) {
                const size_t n = node_index(c, x, y, z);
                double *f = p->f + 27 * n;
                if (!p->fluid[n]) {
                    memset(f, 0, 27 * sizeof(double));
                    continue;
                }
                if (c->init == 1 && c->radius > 0.0) {
                    const double dx = x - axis_x(c), dy = y - axis_y(c);
                    const double u[3] = {0.0, 0.0, loglaw_uz(c, sqrt(dx * dx + dy * dy))};
                    if (c->equilibrium == 1)
                        orc_feq2_r(1.0, u, f);
                    else
                        orc_feq_r(1.0, u, f);
                } else {
                    for (int i = 0; i < 27; ++i) f[i] = ORC_W[i];
                }
            }
}

orc_pipe *orc_pipe_new(const orc_config *cfg, const double *amps)
{
    orc_setup();
    orc_pipe *p = (orc_pipe *)calloc(1, sizeof(orc_pipe));
    if (!p) return NULL;
    p->cfg = *cfg;
    if (p->cfg.n_modes < 0) p->cfg.n_modes = 0;
    if (p->cfg.n_modes > 6) p->cfg.n_modes = 6;
    for (int k = 0; k < 2 * p->cfg.n_modes; ++k) p->amps[k] = amps ? amps[k] : 0.0;
    const orc_config *c = &p->cfg;
    p->nnode = (size_t)c->nx * c->ny * c->nz;
    p->fluid = (uint8_t *)malloc(p->nnode);
    p->f = (double *)malloc(p->nnode * 27 * sizeof(double));
    p->fs = (double *)malloc(p->nnode * 27 * sizeof(double));
    p->shape = (double *)malloc(p->nnode * 3 * sizeof(double));
    if (!p->fluid || !p->f || !p->fs || !p->shape) {
        orc_pipe_free(p);
        return NULL;
    }
    p->nfluid = 0;
    for (int z = 0; z < c->nz; ++z)
        for (int y = 0; y < c->ny; ++y)
            for (int x = 0; x < c->nx; ++x) {
                const size_t n = node_index(c, x, y, z);
                p->fluid[n] = (uint8_t)is_fluid_xy(c, x, y);
                p->nfluid += p->fluid[n];
            }
#pragma omp parallel for schedule(static)
    for (int z = 0; z < c->nz; ++z)
        for (int y = 0; y < c->ny; ++y)
            for (int x = 0; x < c->nx; ++x) {
                const size_t n = node_index(c, x, y, z);
                orc_trigger_shape(c, p->amps, x, y, z, p->shape + 3 * n);
            }
    initial_state(p);
    return p;
}

void orc_pipe_free(orc_pipe *p)
{
    if (!p) return;
    free(p->fluid);
    free(p->f);
    free(p->fs);
    free(p->shape);
    free(p);
}

int64_t orc_pipe_step_index(const orc_pipe *p) { return p->step; }
int64_t orc_pipe_fluid_count(const orc_pipe *p) { return p->nfluid; }
void orc_pipe_fluid_mask(const orc_pipe *p, uint8_t *mask) { memcpy(mask, p->fluid, p->nnode); }

/* body acceleration a(x, n) = h z^ + trigger force */
static void node_force(const orc_pipe *p, size_t n, double tf, double a[3])
{
    a[0] = tf * p->shape[3 * n + 0];
    a[1] = tf * p->shape[3 * n + 1];
    a[2] = p->cfg.accel_z + tf * p->shape[3 * n + 2];
}

void orc_pipe_step(orc_pipe *p, int32_t nsteps)
{
    const orc_config *c = &p->cfg;
    const double omega = 1.0 / c->tau;
    for (int32_t t = 0; t < nsteps; ++t) {
        const double tf = time_factor(c, p->step);
        /* collision at every fluid node */
#pragma omp parallel for schedule(static)
        for (int z = 0; z < c->nz; ++z)
            for (int y = 0; y < c->ny; ++y)
                for (int x = 0; x < c->nx; ++x) {
                    const size_t n = node_index(c, x, y, z);
                    if (!p->fluid[n]) continue;
                    double a[3];
                    node_force(p, n, tf, a);
                    orc_collide_kind_r(p->f + 27 * n, a, omega, c->collision, c->equilibrium, p->fs + 27 * n,
                                       NULL, NULL);
                }
        /* streaming with the wall */
#pragma omp parallel for schedule(static)
        for (int z = 0; z < c->nz; ++z)
            for (int y = 0; y < c->ny; ++y)
                for (int x = 0; x < c->nx; ++x) {
                    const size_t n = node_index(c, x, y, z);
                    if (!p->fluid[n]) continue;
                    for (int i = 0; i < 27; ++i) {
                        size_t src[2];
                        int pop[2];
                        double coef[2];
                        const int nt = stream_terms(p, x, y, z, i, src, pop, coef);
                        double v = 0.0;
                        for (int k = 0; k < nt; ++k) v += coef[k] * p->fs[27 * src[k] + pop[k]];
                        p->f[27 * n + i] = v;
                    }
                }
        p->step += 1;
    }
}

/* Streaming alone (Eq. (streaming) with the wall), applied to the stored
 * state as if it were post-collision: f <- S f.  Used to check that pull
 * streaming with halfway bounce-back is a permutation. */
void orc_pipe_stream(orc_pipe *p)
{
    const orc_config *c = &p->cfg;
    memcpy(p->fs, p->f, p->nnode * 27 * sizeof(double));
    for (int z = 0; z < c->nz; ++z)
        for (int y = 0; y < c->ny; ++y)
            for (int x = 0; x < c->nx; ++x) {
                const size_t n = node_index(c, x, y, z);
                if (!p->fluid[n]) continue;
                for (int i = 0; i < 27; ++i) {
                    size_t src[2];
                    int pop[2];
                    double coef[2];
                    const int nt = stream_terms(p, x, y, z, i, src, pop, coef);
                    double v = 0.0;
                    for (int k = 0; k < nt; ++k) v += coef[k] * p->fs[27 * src[k] + pop[k]];
                    p->f[27 * n + i] = v;
                }
            }
}

void orc_pipe_get_f(const orc_pipe *p, double *out)
{
    for (size_t n = 0; n < p->nnode; ++n)
        for (int i = 0; i < 27; ++i) out[(size_t)i * p->nnode + n] = p->f[27 * n + i];
}

void orc_pipe_set_f(orc_pipe *p, const double *in, int64_t step)
{
    for (size_t n = 0; n < p->nnode; ++n)
        for (int i = 0; i < 27; ++i) p->f[27 * n + i] = p->fluid[n] ? in[(size_t)i * p->nnode + n] : 0.0;
    p->step = step;
}

void orc_pipe_force(const orc_pipe *p, int64_t step, double *a)
{
    const double tf = time_factor(&p->cfg, step);
    for (size_t n = 0; n < p->nnode; ++n) {
        double v[3];
        node_force(p, n, tf, v);
        for (int d = 0; d < 3; ++d) a[(size_t)d * p->nnode + n] = p->fluid[n] ? v[d] : 0.0;
    }
}

/* Eqs. (macroscopic_rho), (macroscopic_u) with a = a(x, n) at the current step */
static void node_moments(const orc_pipe *p, size_t n, double tf, double *rho, double u[3])
{
    const double *f = p->f + 27 * n;
    double r = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < 27; ++i) {
        r += f[i];
        for (int d = 0; d < 3; ++d) j[d] += ORC_C[i][d] * f[i];
    }
    double a[3];
    node_force(p, n, tf, a);
    *rho = r;
    for (int d = 0; d < 3; ++d) u[d] = j[d] / r + 0.5 * a[d];
}

void orc_pipe_moments(const orc_pipe *p, double *rho, double *u)
{
    const double tf = time_factor(&p->cfg, p->step);
    for (size_t n = 0; n < p->nnode; ++n) {
        double r = 0.0, v[3] = {0.0, 0.0, 0.0};
        if (p->fluid[n]) node_moments(p, n, tf, &r, v);
        rho[n] = r;
        for (int d = 0; d < 3; ++d) u[(size_t)d * p->nnode + n] = v[d];
    }
}

void orc_pipe_sums(const orc_pipe *p, double out[4])
{
    out[0] = out[1] = out[2] = out[3] = 0.0;
    for (size_t n = 0; n < p->nnode; ++n) {
        if (!p->fluid[n]) continue;
        for (int i = 0; i < 27; ++i) {
            const double v = p->f[27 * n + i];
            out[0] += v;
            for (int d = 0; d < 3; ++d) out[1 + d] += ORC_C[i][d] * v;
        }
    }
}

double orc_pipe_energy(const orc_pipe *p)
{
    const double tf = time_factor(&p->cfg, p->step);
    double e = 0.0;
    for (size_t n = 0; n < p->nnode; ++n) {
        if (!p->fluid[n]) continue;
        double r, u[3];
        node_moments(p, n, tf, &r, u);
        e += 0.5 * r * u[2] * u[2];
    }
    return e / (double)p->nfluid;
}

int32_t orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---------------------------------------------------------------------- */
/* adjoint of the time-averaged streamwise energy                          */
/* ---------------------------------------------------------------------- */

/* node contribution to E: (1/N_f) 1/2 rho u_z^2, u_z = j_z/rho + a_z/2 */
static cplx energy_node_c(const cplx f[27], cplx az, double inv_nf)
{
    cplx r = 0.0, jz = 0.0;
    for (int i = 0; i < 27; ++i) {
        r += f[i];
        jz += ORC_C[i][2] * f[i];
    }
    const cplx uz = jz / r + 0.5 * az;
    return inv_nf * 0.5 * r * uz * uz;
}

/* a(x, n) as complex, given per-mode unit shapes [node][12][3] */
static void force_c(const orc_pipe *p, const double *mshape, size_t n, double tf, const cplx *amps,
                    cplx a[3])
{
    a[0] = 0.0;
    a[1] = 0.0;
    a[2] = p->cfg.accel_z;
    for (int q = 0; q < 2 * p->cfg.n_modes; ++q)
        for (int d = 0; d < 3; ++d) a[d] += tf * amps[q] * mshape[(n * 12 + q) * 3 + d];
}

static double *mode_shapes(const orc_pipe *p)
{
    const orc_config *c = &p->cfg;
    double *ms = (double *)calloc(p->nnode * 12 * 3, sizeof(double));
    for (int z = 0; z < c->nz; ++z)
        for (int y = 0; y < c->ny; ++y)
            for (int x = 0; x < c->nx; ++x) {
                const size_t n = node_index(c, x, y, z);
                for (int q = 0; q < 2 * c->n_modes; ++q)
                    trigger_mode_cart(c, q, 1.0, x, y, z, ms + (n * 12 + q) * 3);
            }
    return ms;
}

static int in_window(int64_t n, int64_t b, int64_t e) { return n >= b && n < e; }

double orc_objective(const orc_config *cfg, const double *amps, int64_t b, int64_t e)
{
    orc_pipe *p = orc_pipe_new(cfg, amps);
    double J = 0.0;
    for (int64_t n = 0; n < e; ++n) {
        if (in_window(n, b, e)) J += orc_pipe_energy(p);
        if (n + 1 < e) orc_pipe_step(p, 1);
    }
    orc_pipe_free(p);
    return J / (double)(e - b);
}

/* Complex-step tangent: run the whole forward model in complex arithmetic
 * with amps[q] + i h; dJ/d amps[q] = Im J / h. */
double orc_tangent_gradient(const orc_config *cfg, const double *amps, int64_t b, int64_t e, double *grad)
{
    orc_pipe *p = orc_pipe_new(cfg, amps);
    const orc_config *c = &p->cfg;
    const size_t N = p->nnode;
    const double h = 1e-30, omega = 1.0 / c->tau, inv_nf = 1.0 / (double)p->nfluid;
    double *ms = mode_shapes(p);
    cplx *f = (cplx *)malloc(N * 27 * sizeof(cplx));
    cplx *fs = (cplx *)malloc(N * 27 * sizeof(cplx));
    double Jreal = 0.0;
    for (int q = 0; q < 2 * c->n_modes; ++q) {
        cplx ac[12];
        for (int k = 0; k < 12; ++k) ac[k] = (k < 2 * c->n_modes) ? p->amps[k] : 0.0;
        ac[q] += I * h;
        /* initial state is independent of the amplitudes */
        for (size_t n = 0; n < N * 27; ++n) f[n] = p->f[n];
        cplx J = 0.0;
        for (int64_t step = 0; step < e; ++step) {
            const double tf = time_factor(c, step);
            if (in_window(step, b, e)) {
                cplx Es = 0.0;
                for (size_t n = 0; n < N; ++n) {
                    if (!p->fluid[n]) continue;
                    cplx a[3];
                    force_c(p, ms, n, tf, ac, a);
                    Es += energy_node_c(f + 27 * n, a[2], inv_nf);
                }
                J += Es;
            }
            if (step + 1 >= e) break;
#pragma omp parallel for schedule(static)
            for (size_t n = 0; n < N; ++n) {
                if (!p->fluid[n]) continue;
                cplx a[3];
                force_c(p, ms, n, tf, ac, a);
                orc_collide_kind_c(f + 27 * n, a, omega, c->collision, c->equilibrium, fs + 27 * n, NULL, NULL);
            }
#pragma omp parallel for schedule(static)
            for (int z = 0; z < c->nz; ++z)
                for (int y = 0; y < c->ny; ++y)
                    for (int x = 0; x < c->nx; ++x) {
                        const size_t n = node_index(c, x, y, z);
                        if (!p->fluid[n]) continue;
                        for (int i = 0; i < 27; ++i) {
                            size_t src[2];
                            int pop[2];
                            double coef[2];
                            const int nt = stream_terms(p, x, y, z, i, src, pop, coef);
                            cplx v = 0.0;
                            for (int k = 0; k < nt; ++k) v += coef[k] * fs[27 * src[k] + pop[k]];
                            f[27 * n + i] = v;
                        }
                    }
        }
        J /= (double)(e - b);
        grad[q] = cimag(J) / h;
        Jreal = creal(J);
    }
    if (c->n_modes == 0) Jreal = orc_objective(cfg, amps, b, e);
    free(f);
    free(fs);
    free(ms);
    orc_pipe_free(p);
    return Jreal;
}

/* Discrete adjoint (reverse sweep).  Forward: f^{n+1} = S C(f^n, a^n).
 *   lambda^{e-1} = dJ/df^{e-1}
 *   mu = S^T lambda^{n+1};  lambda^n = (dC/df)^T mu + dJ/df^n
 *   dJ/d amps[q] += sum_x [(dC/da)^T mu + dJ/da^n] . da^n/d amps[q]
 * Node Jacobians of C and of the energy come from complex-step
 * differentiation of the same formulas the forward run uses. */
double orc_adjoint_gradient(const orc_config *cfg, const double *amps, int64_t b, int64_t e, double *grad)
{
    orc_pipe *p = orc_pipe_new(cfg, amps);
    const orc_config *c = &p->cfg;
    const size_t N = p->nnode;
    const double h = 1e-30, omega = 1.0 / c->tau, inv_nf = 1.0 / (double)p->nfluid;
    const double Wn = 1.0 / (double)(e - b);
    const int nq = 2 * c->n_modes;
    double *ms = mode_shapes(p);
    double *states = (double *)malloc((size_t)e * N * 27 * sizeof(double));
    double J = 0.0;
    for (int64_t n = 0; n < e; ++n) {
        memcpy(states + (size_t)n * N * 27, p->f, N * 27 * sizeof(double));
        if (in_window(n, b, e)) J += orc_pipe_energy(p);
        if (n + 1 < e) orc_pipe_step(p, 1);
    }
    J *= Wn;
    for (int q = 0; q < nq; ++q) grad[q] = 0.0;
    double *lam = (double *)calloc(N * 27, sizeof(double));
    double *mu = (double *)calloc(N * 27, sizeof(double));
    cplx ampc[12];
    for (int k = 0; k < 12; ++k) ampc[k] = (k < nq) ? p->amps[k] : 0.0;

    for (int64_t n = e - 1; n >= 0; --n) {
        const double tf = time_factor(c, n);
        const double *fn = states + (size_t)n * N * 27;
        /* mu = S^T lambda^{n+1} (zero at the last state, which is not collided) */
        memset(mu, 0, N * 27 * sizeof(double));
        if (n + 1 < e) {
            for (int z = 0; z < c->nz; ++z)
                for (int y = 0; y < c->ny; ++y)
                    for (int x = 0; x < c->nx; ++x) {
                        const size_t nd = node_index(c, x, y, z);
                        if (!p->fluid[nd]) continue;
                        for (int i = 0; i < 27; ++i) {
                            size_t src[2];
                            int pop[2];
                            double coef[2];
                            const int nt = stream_terms(p, x, y, z, i, src, pop, coef);
                            for (int k = 0; k < nt; ++k) mu[27 * src[k] + pop[k]] += coef[k] * lam[27 * nd + i];
                        }
                    }
        }
        double gq[12] = {0};
        for (size_t nd = 0; nd < N; ++nd) {
            double *ln = lam + 27 * nd;
            if (!p->fluid[nd]) {
                memset(ln, 0, 27 * sizeof(double));
                continue;
            }
            const double *f = fn + 27 * nd;
            const double *m = mu + 27 * nd;
            cplx a[3];
            force_c(p, ms, nd, tf, ampc, a);
            cplx fc[27], out[27];
            for (int i = 0; i < 27; ++i) fc[i] = f[i];
            double sa[3] = {0.0, 0.0, 0.0}; /* sensitivity to a(x, n) */
            for (int j = 0; j < 27; ++j) {
                double v = 0.0;
                if (n + 1 < e) {
                    fc[j] += I * h;
                    orc_collide_kind_c(fc, a, omega, c->collision, c->equilibrium, out, NULL, NULL);
                    fc[j] = f[j];
                    for (int k = 0; k < 27; ++k) v += cimag(out[k]) / h * m[k];
                }
                if (in_window(n, b, e)) {
                    fc[j] += I * h;
                    v += Wn * cimag(energy_node_c(fc, a[2], inv_nf)) / h;
                    fc[j] = f[j];
                }
                ln[j] = v;
            }
            for (int d = 0; d < 3; ++d) {
                cplx ad[3] = {a[0], a[1], a[2]};
                ad[d] += I * h;
                if (n + 1 < e) {
                    orc_collide_kind_c(fc, ad, omega, c->collision, c->equilibrium, out, NULL, NULL);
                    for (int k = 0; k < 27; ++k) sa[d] += cimag(out[k]) / h * m[k];
                }
                if (d == 2 && in_window(n, b, e)) sa[d] += Wn * cimag(energy_node_c(fc, ad[2], inv_nf)) / h;
            }
            for (int q = 0; q < nq; ++q)
                for (int d = 0; d < 3; ++d) gq[q] += sa[d] * tf * ms[(nd * 12 + q) * 3 + d];
        }
        for (int q = 0; q < nq; ++q) grad[q] += gq[q];
    }
    free(lam);
    free(mu);
    free(states);
    free(ms);
    orc_pipe_free(p);
    return J;
}
