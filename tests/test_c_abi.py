"""The C-ABI from C (CPU only, no GPU): a C99 program compiled with -Werror
against include/lbm.h and linked to the built liblbm.so calls the host-only
entry points.  It checks the layout of the turbulent pipe (192 x 192 x 1152,
R = 90: 25,448 fluid columns, the same count the Python binding and the
oracle give), that the workspace holds at least the two state buffers, and
that invalid configurations return LBM_EINVAL without touching the output.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBDIR = os.path.join(ROOT, "paper_2405_12082_amd")

PROGRAM = r"""
#include <stdio.h>
#include <string.h>
#include "lbm.h"

static lbm_config base(void)
{
    lbm_config c;
    memset(&c, 0, sizeof c);
    c.nx = 192; c.ny = 192; c.nz = 1152; c.batch = 1;
    c.radius = 90.0; c.tau = 0.505778; c.accel_z = 1.0e-6;
    c.kz = 3.0; c.kappa = 0.5; c.l0_frac = 0.2; c.l_frac = 0.4;
    return c;
}

int main(void)
{
    lbm_config c = base();
    lbm_layout lay;
    size_t ws = 0;
    if (lbm_describe(&c, &lay) != LBM_OK) return 10;
    if (lbm_workspace_bytes(&c, &ws) != LBM_OK) return 11;
    printf("%lld %lld %lld %lld %lld %lld %zu\n", (long long)lay.n_fluid_columns, (long long)lay.plane_pitch,
           (long long)lay.n_fluid_nodes, (long long)lay.state_bytes, (long long)lay.bytes_per_update,
           (long long)lay.population_stride, ws);
    /* invalid configurations: LBM_EINVAL, output untouched */
    lbm_layout bad;
    memset(&bad, 0x5a, sizeof bad);
    lbm_config t = base();
    t.tau = 0.5;
    if (lbm_describe(&t, &bad) != LBM_EINVAL) return 20;
    t = base();
    t.storage = 3;
    if (lbm_describe(&t, &bad) != LBM_EINVAL) return 21;
    t = base();
    t.wall = 1;
    t.pattern = 1;
    if (lbm_describe(&t, &bad) != LBM_EINVAL) return 22;
    if (lbm_describe(NULL, &bad) != LBM_EINVAL) return 23;
    const unsigned char *pb = (const unsigned char *)&bad;
    for (size_t i = 0; i < sizeof bad; ++i)
        if (pb[i] != 0x5a) return 24;
    return 0;
}
"""


def test_header_compiles_as_c_and_host_calls_work(tmp_path):
    cc = shutil.which("gcc") or shutil.which("cc")
    lib = os.path.join(LIBDIR, "liblbm.so")
    if not cc:
        pytest.skip("no C compiler")
    if not os.path.exists(lib):
        pytest.skip("liblbm.so not built")
    src = tmp_path / "abi.c"
    exe = tmp_path / "abi"
    src.write_text(PROGRAM)
    subprocess.run([cc, "-std=c99", "-Wall", "-Wextra", "-Werror", "-I", os.path.join(ROOT, "include"), str(src),
                    "-o", str(exe), "-L", LIBDIR, "-llbm", f"-Wl,-rpath,{LIBDIR}"], check=True)
    res = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert res.returncode == 0, (res.returncode, res.stderr)
    ncol, pitch, nodes, state, bpu, pstride, ws = map(int, res.stdout.split())
    assert ncol == 25448 and nodes == 25448 * 1152
    assert pitch % 64 == 0 and pitch >= ncol
    assert pstride >= 1152 * pitch and pstride % 64 == 0
    assert bpu == 216
    assert state >= 4 * 27 * pstride
    assert ws >= 2 * state
