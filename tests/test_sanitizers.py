"""CPU sanitizer builds (no GPU): the FP64 oracle and the host side of the
HIP library's runtime under AddressSanitizer and UndefinedBehaviorSanitizer.

* The oracle (C11 + OpenMP) is compiled with gcc -fsanitize=address,undefined
  into a driver that calls every exported function: the per-node formulas
  (real and complex step), every collision kind, pipes with both walls, all
  collision kinds and the trigger force, moments, sums, energy, the adjoint
  and the tangent gradient on a tiny pipe.
* The library is compiled with the sanitizers on its host code only
  (device code is unaffected), and a C driver built with the same compiler
  calls the host-only entry points over valid and invalid configurations
  (layout construction, validation, the two-step tile tables, workspace
  carving).
Any report makes the driver exit non-zero (-fno-sanitize-recover)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

ORACLE_DRIVER = r"""
#include <math.h>
#include <stdio.h>
#include <string.h>
#include "lbm_oracle.h"

static int bad(const double *v, int n)
{
    for (int i = 0; i < n; ++i)
        if (!isfinite(v[i])) return 1;
    return 0;
}

int main(void)
{
    int32_t c[81], opp[27];
    double w[27], A[729], Ai[729], f[27], fs[27], m[27], R[27], F[27];
    orc_lattice(c, w, opp);
    orc_moment_matrix(A);
    orc_moment_matrix_inverse(Ai);
    const double u[3] = {0.02, -0.01, 0.05}, a[3] = {1e-4, -2e-4, 3e-4};
    orc_feq(1.01, u, f);
    orc_meq(1.01, u, m);
    orc_rmrt(1.01, u, a, R);
    orc_feq2(1.01, u, fs);
    orc_force2(1.01, u, a, F);
    if (bad(f, 27) || bad(m, 27) || bad(R, 27) || bad(fs, 27) || bad(F, 27)) return 2;
    for (int coll = 0; coll < 2; ++coll)
        for (int eq = 0; eq < 2; ++eq) {
            orc_collide_kind(f, a, 1.7, coll, eq, fs);
            if (bad(fs, 27)) return 3;
        }
    orc_collide(f, a, 1.7, fs);
    double rc[2] = {1.0, 1e-30}, uc[6] = {0.02, 0, -0.01, 0, 0.05, 1e-30}, fc[54], ac[6] = {1e-4, 0, 0, 0, 0, 0};
    orc_feq_cplx(rc, uc, fc);
    orc_meq_cplx(rc, uc, fc);
    double fin[54];
    for (int i = 0; i < 27; ++i) { fin[2 * i] = f[i]; fin[2 * i + 1] = 0.0; }
    orc_collide_cplx(fin, ac, 1.7, fc);
    if (bad(fc, 54)) return 4;
    orc_config cfg;
    memset(&cfg, 0, sizeof cfg);
    cfg.nx = 12; cfg.ny = 11; cfg.nz = 5; cfg.radius = 4.7; cfg.tau = 0.6; cfg.accel_z = 1e-5;
    cfg.n_modes = 2; cfg.kz = 1.0; cfg.kappa = 0.5; cfg.l0_frac = 0.2; cfg.l_frac = 0.4; cfg.period = 10.0;
    cfg.force_off_step = 100; cfg.init = 1; cfg.u_tau = 0.01;
    const double amps[4] = {1e-4, 2e-4, -1e-4, 5e-5};
    double out[3];
    orc_trigger_shape(&cfg, amps, 3.0, 4.0, 1.0, out);
    orc_force_at(&cfg, amps, 3, 4, 1, 2, out);
    (void)orc_bouzidi(0.3, 0.1, 0.2, 0.05, 1);
    (void)orc_bouzidi(0.7, 0.1, 0.2, 0.05, 0);
    for (int wall = 0; wall < 2; ++wall)
        for (int kind = 0; kind < 4; ++kind) {
            cfg.wall = wall;
            cfg.collision = kind >> 1;
            cfg.equilibrium = kind & 1;
            orc_pipe *p = orc_pipe_new(&cfg, amps);
            if (!p) return 5;
            (void)orc_wall_fraction(&cfg, 9, 5, 1);
            orc_pipe_step(p, 3);
            orc_pipe_stream(p);
            const size_t n = (size_t)cfg.nx * cfg.ny * cfg.nz;
            static double buf[27 * 12 * 11 * 5], rho[12 * 11 * 5], uu[3 * 12 * 11 * 5];
            static uint8_t mask[12 * 11 * 5];
            orc_pipe_get_f(p, buf);
            orc_pipe_set_f(p, buf, 3);
            orc_pipe_force(p, 3, uu);
            orc_pipe_moments(p, rho, uu);
            orc_pipe_fluid_mask(p, mask);
            double sums[4];
            orc_pipe_sums(p, sums);
            const double e = orc_pipe_energy(p);
            if (bad(buf, (int)(27 * n)) || bad(sums, 4) || !isfinite(e)) return 6;
            if (orc_pipe_step_index(p) != 3 || orc_pipe_fluid_count(p) <= 0) return 7;
            orc_pipe_free(p);
        }
    cfg.wall = 1;
    cfg.collision = 0;
    cfg.equilibrium = 0;
    double g1[4], g2[4];
    const double J1 = orc_adjoint_gradient(&cfg, amps, 2, 5, g1);
    const double J2 = orc_tangent_gradient(&cfg, amps, 2, 5, g2);
    const double J3 = orc_objective(&cfg, amps, 2, 5);
    if (bad(g1, 4) || bad(g2, 4) || !isfinite(J1 + J2 + J3)) return 8;
    printf("ok %d threads\n", orc_num_threads());
    return 0;
}
"""

LIBRARY_DRIVER = r"""
#include <stdio.h>
#include <string.h>
#include "lbm.h"

static lbm_config base(void)
{
    lbm_config c;
    memset(&c, 0, sizeof c);
    c.nx = 40; c.ny = 36; c.nz = 20; c.batch = 2;
    c.radius = 16.5; c.tau = 0.55; c.accel_z = 1.0e-6; c.n_modes = 3; c.period = 30.0;
    c.kz = 3.0; c.kappa = 0.5; c.l0_frac = 0.2; c.l_frac = 0.4; c.force_off_step = 50;
    c.init = 1; c.u_tau = 0.01;
    return c;
}

int main(void)
{
    lbm_layout lay;
    size_t ws;
    int valid = 0, invalid = 0;
    for (int storage = 0; storage < 4; ++storage)
        for (int wall = 0; wall < 3; ++wall)
            for (int pattern = 0; pattern < 2; ++pattern)
                for (int adj = 0; adj < 3; ++adj)
                    for (int kind = 0; kind < 4; ++kind)
                        for (int shape = 0; shape < 4; ++shape) {
                            lbm_config c = base();
                            c.storage = storage; c.wall = wall; c.pattern = pattern; c.adjoint = adj;
                            c.collision = kind >> 1; c.equilibrium = kind & 1;
                            if (shape == 1) { c.radius = 0.0; c.n_modes = 0; c.init = 0; c.nx = 3; c.ny = 2; }
                            if (shape == 2) { c.nx = 300; c.ny = 300; c.nz = 4; c.radius = 149.5; c.batch = 1; }
                            if (shape == 3) { c.block = 64; c.zchunk = 64; c.xcd_remap = 4096; }
                            const int r1 = lbm_describe(&c, &lay), r2 = lbm_workspace_bytes(&c, &ws);
                            if (r1 != r2) return 10;
                            if (r1 == LBM_OK) {
                                ++valid;
                                if (ws < (size_t)lay.state_bytes || lay.n_fluid_columns <= 0) return 11;
                            } else if (r1 == LBM_EINVAL) {
                                ++invalid;
                            } else {
                                return 12;
                            }
                        }
    lbm_config c = base();
    c.tau = 0.5;
    if (lbm_describe(&c, &lay) != LBM_EINVAL) return 13;
    if (lbm_describe(NULL, &lay) != LBM_EINVAL) return 14;
    if (lbm_set_watchdog(NULL, 1e-6) != LBM_EINVAL) return 15;
    if (lbm_get_step(NULL, NULL) != LBM_EINVAL) return 16;
    if (lbm_ring_spectrum_static(NULL, 1, 1, 64, 4, NULL, NULL, NULL, NULL) != LBM_EINVAL) return 17;
    if (lbm_recompute_moments(NULL, NULL, 0, 1, NULL, 0, NULL, 0) != LBM_EINVAL) return 19;
    if (lbm_adjoint_step_moments(NULL, 1, NULL, 0, NULL) != LBM_EINVAL) return 20;
    if (lbm_step_recording(NULL, 1, NULL, 0) != LBM_EINVAL) return 22;
    lbm_config r = base();
    r.adjoint = 1;
    lbm_layout rl;
    if (lbm_describe(&r, &rl) != LBM_OK || rl.record_bytes < 4 * 4 * rl.n_fluid_nodes * r.batch) return 21;
    printf("%d %d\n", valid, invalid);
    return valid > 0 && invalid > 0 ? 0 : 18;
}
"""

SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def test_oracle_under_asan_ubsan(tmp_path):
    cc = shutil.which("gcc")
    if not cc:
        pytest.skip("no gcc")
    src = tmp_path / "oracle_driver.c"
    exe = tmp_path / "oracle_driver"
    src.write_text(ORACLE_DRIVER)
    odir = os.path.join(ROOT, "oracle")
    subprocess.run([cc, "-std=gnu11", "-O1", "-g", "-fopenmp", *SAN, "-I", odir, str(src),
                    os.path.join(odir, "lbm_oracle.c"), "-o", str(exe), "-lm"], check=True)
    env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600, env=env)
    assert res.returncode == 0, (res.returncode, res.stdout[-2000:], res.stderr[-4000:])
    assert res.stdout.startswith("ok")


def test_library_host_code_under_asan_ubsan(tmp_path):
    """The library's host code with the sanitizers (hipcc, which instruments
    only the host side here), driven from C through the host-only calls."""
    hipcc = shutil.which("hipcc")
    clang = "/opt/rocm/llvm/bin/clang"
    if not hipcc or not os.path.exists(clang):
        pytest.skip("no hipcc / clang")
    import sys
    sys.path.insert(0, os.path.join(ROOT, "paper_2405_12082_amd"))
    import build as B
    csrc = os.path.join(ROOT, "paper_2405_12082_amd", "csrc")
    host_san = []
    for flag in SAN:
        host_san += ["-Xarch_host", flag]
    objs, procs = [], []
    for s in B.SOURCES:
        o = str(tmp_path / (os.path.splitext(s)[0] + ".o"))
        procs.append(subprocess.Popen([hipcc, *B.hipcc_flags(), *host_san, "-g", "-c", os.path.join(csrc, s), "-o", o],
                                      stdout=subprocess.DEVNULL, stderr=subprocess.PIPE))
        objs.append(o)
    for p in procs:
        _, err = p.communicate(timeout=900)
        assert p.returncode == 0, err.decode()[-2000:]
    lib = str(tmp_path / "liblbm_san.so")
    subprocess.run([hipcc, "--offload-arch=" + B.ARCH, "-shared", "-fPIC", *host_san, "-o", lib, *objs], check=True,
                   stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    src = tmp_path / "lib_driver.c"
    exe = tmp_path / "lib_driver"
    src.write_text(LIBRARY_DRIVER)
    subprocess.run([clang, "-std=c99", "-g", *SAN, "-I", os.path.join(ROOT, "include"), str(src), lib,
                    f"-Wl,-rpath,{tmp_path}", "-o", str(exe)], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert res.returncode == 0, (res.returncode, res.stdout[-2000:], res.stderr[-4000:])
    valid, invalid = map(int, res.stdout.split())
    assert valid > 50 and invalid > 50
