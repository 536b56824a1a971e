"""Host-side checks of the HIP library (no GPU needed): it loads, exports
every function include/lbm.h declares, and its configuration checks and
layout reports are right."""
import ctypes as C

import numpy as np
import pytest

import lbm_inputs as LI
import paper_2405_12082_amd as P
from paper_2405_12082_amd import _lib


def test_library_exports_every_header_function():
    names = P.header_functions()
    assert len(names) >= 20
    L = P.lib()
    for n in names:
        assert hasattr(L, n), n


@pytest.mark.parametrize("name,ncol,nodes", [
    ("laminar", 316, 15168),
    ("turbulent", 25448, 29316096),
    ("precision_ref", 2828, 723968),
    ("batched", 2828, 723968),
    ("adjoint", 6376, 2448384),
    ("paper", 70168, 42100800),
])
def test_layout_counts_fluid_columns(name, ncol, nodes, oracle_mod):
    cfg = LI.preset(name)
    lay = P.describe(P.make_config(**cfg))
    assert lay.n_fluid_columns == ncol
    assert lay.n_fluid_nodes == nodes
    assert lay.plane_pitch % 64 == 0 and lay.plane_pitch >= ncol
    assert lay.bytes_per_update == 216
    ps = lay.population_stride
    assert ps % 64 == 0 and ps >= cfg["nz"] * lay.plane_pitch
    assert ps % 4096 != 0  # streams of a step not aligned modulo 16 KiB (FP32)
    assert ps - cfg["nz"] * lay.plane_pitch in (0, 2368)
    assert lay.state_bytes >= 4 * 27 * ps * cfg["batch"]
    if name == "laminar":
        # same fluid set as the oracle's mask
        o = oracle_mod.Pipe(oracle_mod.make_config(**cfg))
        assert o.fluid_mask()[0].sum() == ncol


def test_fp16_storage_halves_the_state():
    cfg = LI.preset("turbulent")
    a = P.describe(P.make_config(**cfg))
    cfg["storage"] = 1
    b = P.describe(P.make_config(**cfg))
    assert b.bytes_per_update == 108
    assert abs(b.state_bytes * 2 - a.state_bytes) <= 512


@pytest.mark.parametrize("bad", [
    dict(nx=0), dict(batch=0), dict(tau=0.5), dict(tau=0.4), dict(n_modes=7), dict(n_modes=-1),
    dict(storage=3), dict(storage=2, adjoint=1), dict(adjoint=3), dict(wall=2), dict(wall=1, pattern=1),
    dict(wall=1, radius=0.0), dict(pattern=2),
    dict(pattern=1, adjoint=1),
    dict(init=2), dict(radius=12.0),
    dict(block=96), dict(zchunk=65), dict(n_modes=2, period=0.0), dict(radius=0.4),
])
def test_invalid_configurations_are_rejected(bad):
    cfg = LI.preset("laminar")
    cfg.update(bad)
    c = P.make_config(**cfg)
    out = _lib.LbmLayout()
    assert P.lib().lbm_describe(C.byref(c), C.byref(out)) == _lib.LBM_EINVAL
    nbytes = C.c_size_t(0)
    assert P.lib().lbm_workspace_bytes(C.byref(c), C.byref(nbytes)) == _lib.LBM_EINVAL


def test_null_arguments():
    L = P.lib()
    assert L.lbm_describe(None, None) == _lib.LBM_EINVAL
    ctx = C.c_void_p()
    cfg = P.make_config(**LI.preset("laminar"))
    # no workspace -> rejected before any device call
    assert L.lbm_init(C.byref(cfg), None, None, 0, None, C.byref(ctx)) == _lib.LBM_ENOMEM
    assert ctx.value is None
    assert L.lbm_step(None, 1) == _lib.LBM_EINVAL
    assert L.lbm_last_error(None) == b"no context"


def test_workspace_grows_with_adjoint_buffers():
    cfg = LI.preset("adjoint")
    a = P.describe(P.make_config(**cfg)).workspace_bytes
    cfg["adjoint"] = 1
    b = P.describe(P.make_config(**cfg)).workspace_bytes
    assert b - a >= 2 * 4 * 27 * 384 * 6400


def test_aa_pattern_keeps_one_state_buffer():
    cfg = LI.preset("turbulent")
    ab = P.describe(P.make_config(**cfg))
    cfg["pattern"] = 1
    aa = P.describe(P.make_config(**cfg))
    assert aa.state_bytes == ab.state_bytes and aa.bytes_per_update == ab.bytes_per_update
    assert ab.workspace_bytes - aa.workspace_bytes == ab.state_bytes


def test_interpolated_wall_is_a_valid_configuration():
    cfg = LI.preset("laminar")
    a = P.describe(P.make_config(**cfg))
    cfg["wall"] = 1
    b = P.describe(P.make_config(**cfg))
    assert b.n_fluid_nodes == a.n_fluid_nodes
    assert b.workspace_bytes - a.workspace_bytes >= 9 * b.plane_pitch * 8  # coefficient table


def test_periodic_box_layout():
    lay = P.describe(P.make_config(nx=1, ny=1, nz=64, radius=0.0, tau=0.8))
    assert lay.n_fluid_columns == 1 and lay.n_fluid_nodes == 64


def test_counter_based_generator_matches_sequential():
    a = LI.uniform01(11, 50)
    b = LI.hash_uniform(11, np.arange(50))
    assert np.array_equal(a, b)


def test_population_size_limit():
    """The kernels address one population's region with 32-bit byte offsets:
    a population of the state (or of the adjoint state) must take < 4 GiB."""
    def rc(**kw):
        cfg = dict(LI.preset("turbulent"), nx=512, ny=512, radius=255.5, **kw)
        return P.lib().lbm_describe(C.byref(P.make_config(**cfg)), C.byref(_lib.LbmLayout()))
    # about 205,000 fluid columns: 4000 planes take 3.3 GB per FP32 population
    assert rc(nz=4000) == _lib.LBM_OK
    assert rc(nz=4000, adjoint=1) == _lib.LBM_OK
    assert rc(nz=4000, adjoint=2) == _lib.LBM_EINVAL   # 6.6 GB per FP64 adjoint population
    assert rc(nz=4000, storage=2) == _lib.LBM_EINVAL   # FP64 state
    assert rc(nz=6000) == _lib.LBM_EINVAL
    assert rc(nz=6000, storage=1) == _lib.LBM_OK       # FP16: 2.5 GB
    assert rc(nz=6000, storage=1, adjoint=1) == _lib.LBM_EINVAL
