"""The checked build (needs an MI355X).

liblbm_checked.so is built from the same sources with the device-side
bounds tests compiled in (include/lbm.h, lbm_check_flags): every population
load and store of the gather and store paths, every neighbour-table entry
and column index.  Run on every kernel path -- both patterns, both walls,
the three storage forms, batched and persistent launches, graph replay, two
steps per launch, the comparison schemes, the observers and the coherent-
structure sampling, the adjoint with recomputation (moment records and
saved states, FP32 and FP16 forward) -- it records no
violation, and its results equal the release build's bitwise (the tests
change no arithmetic)."""
import sys

import numpy as np
import pytest

import lbm_inputs as LI

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def libs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2405_12082_amd import _lib
    return _lib.lib(), _lib.checked_lib()


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _cfg(**kw):
    cfg = dict(nx=26, ny=24, nz=12, batch=1, radius=11.3, tau=0.56, accel_z=3e-6, n_modes=3, kz=3.0, kappa=0.5,
               l0_frac=0.2, l_frac=0.4, period=30.0, force_off_step=1000, storage=0, wall=0, pattern=0, init=1,
               u_tau=0.01)
    cfg.update(kw)
    return cfg


def _amps(cfg):
    return LI.batch_amplitudes(3, cfg["batch"], cfg["n_modes"], cfg["u_tau"], cfg["period"]) * 10.0


def _both(libs, cfg, run):
    """run(pipe) -> dict of arrays, on the release and the checked build;
    the checked one records no violation and both agree bitwise."""
    import paper_2405_12082_amd as P
    out = []
    for k, lib in enumerate(libs):
        p = P.Pipe(cfg, _amps(cfg), library=lib)
        res = run(p)
        flags, checked = p.check_flags()
        assert checked == (k == 1)
        assert flags == 0, f"bounds-check flags {flags:#x}"
        out.append({name: np.asarray(v.cpu() if hasattr(v, "cpu") else v) for name, v in res.items()})
        p.close()
    for name in out[0]:
        assert np.array_equal(out[0][name], out[1][name], equal_nan=True), name


def _state(p):
    return {"pops": p.populations()}


@pytest.mark.parametrize("storage", [0, 1, 2])
@pytest.mark.parametrize("wall", [0, 1])
@pytest.mark.parametrize("pattern", [0, 1])
def test_steps_graphs_and_observers(libs, storage, wall, pattern):
    if pattern == 1 and wall == 1:
        pytest.skip("the AA pattern has the bounce-back wall only")
    _log(f"checked build: storage {storage} wall {wall} pattern {pattern}")
    cfg = _cfg(storage=storage, wall=wall, pattern=pattern, block=64, zchunk=5)

    def run(p):
        p.step(7)
        p.step_graph(8, 4)
        rho, u = p.moments()
        p.profile_accumulate()
        r = {"pops": p.populations(), "rho": rho, "u": u, "diag": p.diagnostics(), "energy": p.energy(),
             "prof": p.profile_read()}
        ring = p.ring_sample(0.78 * cfg["radius"], 64)
        _, mean, dom = p.ring_spectrum(ring, 8)
        r.update(ring=ring, mean=mean, dom=dom)
        return r
    _both(libs, cfg, run)


@pytest.mark.parametrize("pattern", [0, 1])
def test_batched_and_persistent_launches(libs, pattern):
    cfg = _cfg(batch=3, pattern=pattern)

    def run(p):
        p.set_launch(block=128, zchunk=3, xcd_remap=1, pipes_per_launch=2, pipe_major=1)
        p.step_graph(6, 2)
        p.step_persistent(5)
        p.step_persistent_graph(8, 4)
        return _state(p)
    _both(libs, cfg, run)


@pytest.mark.parametrize("storage", [0, 1])
def test_two_steps_per_launch(libs, storage):
    cfg = _cfg(storage=storage, nz=20)

    def run(p):
        p.set_fused(2, 8)
        p.step(7)
        return _state(p)
    _both(libs, cfg, run)


@pytest.mark.parametrize("kind", [(0, 1), (1, 0), (1, 1)])
@pytest.mark.parametrize("wall", [0, 1])
def test_comparison_schemes(libs, kind, wall):
    cfg = _cfg(collision=kind[0], equilibrium=kind[1], wall=wall)

    def run(p):
        p.step(9)
        return _state(p)
    _both(libs, cfg, run)


@pytest.mark.parametrize("records", ["moments", "states", "recorded forward"])
@pytest.mark.parametrize("storage", [0, 1])
@pytest.mark.parametrize("wall", [0, 1])
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_adjoint_with_recompute(libs, wall, precision, storage, records):
    from paper_2405_12082_amd.adjoint import EnergyAdjoint
    cfg = _cfg(wall=wall, nz=16, storage=storage)
    grads = []
    for lib in libs:
        if records == "recorded forward":
            run = EnergyAdjoint(cfg, 20, 40, precision=precision, library=lib, recompute=False)
        else:
            run = EnergyAdjoint(cfg, 20, 40, checkpoint_every=10, precision=precision, library=lib, records=records)
        J, g = run.gradient(_amps(cfg))
        flags, checked = run.pipe.check_flags()
        assert flags == 0, f"bounds-check flags {flags:#x}"
        grads.append((J, g))
    assert np.array_equal(grads[0][0], grads[1][0]) and np.array_equal(grads[0][1], grads[1][1])


def test_a_corrupt_neighbour_entry_is_caught(libs):
    """A neighbour-table entry pointing far outside the table, planted from
    the host in the checked build's workspace (FP32 storage, two buffers: the
    step kernel reads the table only through its checked gather set-up): the
    step flags it (bit 1) and uses the column itself instead of reading
    outside the state; the step still completes."""
    import paper_2405_12082_amd as P
    cfg = _cfg()
    p = P.Pipe(cfg, _amps(cfg), library=libs[1])
    ncol, pitch = int(p.layout.n_fluid_columns), int(p.layout.plane_pitch)
    ws = p.workspace.view(torch.int32)
    ar = torch.arange(ncol, dtype=torch.int32, device=ws.device)
    # the table is [9][pitch] int32; row 4 (the column itself) reads 0, 1, ..., ncol - 1
    cand = torch.nonzero((ws[:-2] == 0) & (ws[1:-1] == 1) & (ws[2:] == 2)).flatten().tolist()
    rows = [j for j in cand if j + ncol <= ws.numel() and bool(torch.equal(ws[j:j + ncol], ar))]
    assert len(rows) == 1, rows
    base = rows[0] - 4 * pitch
    assert base >= 0
    torch.cuda.synchronize()
    ws[base] = 1 << 30  # row 0 (neighbour (-1, -1)) of column 0
    torch.cuda.synchronize()
    assert p.check_flags() == (0, True)
    p.step(1)
    flags, _ = p.check_flags()
    assert flags & 1 and not flags & ~1, f"{flags:#x}"
    p.close()


def test_checked_build_on_a_pipe_beyond_2_31_elements(libs):
    """The checked build on a pipe of more than 2^31 state elements (384^2 x
    1024, R = 180, FP16 and FP32): no violation in 3 steps, and the state
    equals the release build's bitwise (compared on the device)."""
    import paper_2405_12082_amd as P
    for storage in (1, 0):
        cfg = dict(LI.preset("turbulent"), nx=384, ny=384, nz=1024, radius=180.0, storage=storage)
        _log(f"checked build, 384^2 x 1024 pipe, storage {storage}")
        ref = None
        for k, lib in enumerate(libs):
            p = P.Pipe(cfg, LI.preset_amplitudes(cfg), library=lib)
            p.step(3)
            flags, checked = p.check_flags()
            assert flags == 0 and checked == (k == 1), (flags, checked)
            g = p.populations()
            p.close()
            del p
            if ref is None:
                ref = g
            else:
                assert torch.equal(ref, g)
            del g
            torch.cuda.empty_cache()
        del ref
        torch.cuda.empty_cache()
