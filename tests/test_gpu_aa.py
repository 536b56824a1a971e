"""The in-place AA pattern (one buffer; even steps read and write a node's
own slots, odd steps its neighbours') on the GPU (needs an MI355X).

Per node it gathers the same values and runs the same collision as the
two-buffer pattern, so from the same state its states are bitwise equal to
the two-buffer states at every step and for every storage; one step from a
random state at an even and at an odd step index is also checked against
the FP64 oracle directly.
"""
import sys

import numpy as np
import pytest

import lbm_inputs as LI

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2405_12082_amd as P
    P.lib()
    return P


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _cfg(**kw):
    cfg = dict(nx=21, ny=23, nz=13, batch=1, radius=9.6, tau=0.56, accel_z=3e-6, n_modes=6,
               kz=3.0, kappa=0.5, l0_frac=0.2, l_frac=0.4, period=40.0, force_off_step=1000,
               storage=0, wall=0, pattern=0, init=1, u_tau=0.01)
    cfg.update(kw)
    return cfg


def _amps(cfg, seed=5, boost=1.0):
    return LI.batch_amplitudes(seed, cfg["batch"], cfg["n_modes"], cfg["u_tau"], cfg["period"]) * boost


def _pops(p):
    return p.populations().cpu().numpy()


@pytest.mark.parametrize("s0,zchunk,block,nz", [(10, 4, 256, 13), (11, 4, 256, 13), (11, 1, 64, 13), (10, 5, 128, 13),
                                                (10, 1, 256, 1), (11, 1, 256, 1), (10, 2, 128, 2), (11, 1, 64, 2)])
def test_aa_single_step_random_state_vs_oracle(P, oracle_mod, s0, zchunk, block, nz):
    """One step from seeded random deviations written at an even (own slots)
    or odd (exchanged slots) step index: every population of every fluid
    node matches the oracle's collide + stream, within
    64 * 2^-24 * (max|g_in| + max|g_out|); also on pipes of one and two
    planes (the odd step's pushes along z land in the same or the other
    plane)."""
    O = oracle_mod
    cfg = _cfg(pattern=1, zchunk=zchunk, block=block, nz=nz)
    amps = _amps(cfg, boost=40.0)
    _log(f"AA single step s0={s0} zchunk={zchunk} block={block} nz={nz}")
    mask = O.Pipe(O.make_config(**cfg)).fluid_mask()
    g0 = LI.random_deviations(321, (cfg["nz"], cfg["ny"], cfg["nx"]))
    g0[:, ~mask] = 0.0
    p = P.Pipe(cfg, amps)
    p.set_populations(torch.from_numpy(g0[None]).cuda(), step=s0)
    assert np.array_equal(_pops(p)[0], g0), "set/get populations must round-trip exactly"
    p.step(1)
    g1 = _pops(p)[0].astype(np.float64)
    o = O.Pipe(O.make_config(**cfg), amps[0])
    _, w, _ = O.lattice()
    f0 = g0.astype(np.float64) + w[:, None, None, None]
    f0[:, ~mask] = 0.0
    o.set_f(f0, s0)
    o.step(1)
    go = o.get_f() - w[:, None, None, None]
    tol = 64 * 2.0 ** -24 * (np.abs(g0).max() + np.abs(go[:, mask]).max())
    err = np.abs(g1[:, mask] - go[:, mask]).max()
    _log(f"max abs error {err:.3e} (tolerance {tol:.3e})")
    assert err <= tol
    assert np.all(g1[:, ~mask] == 0)


def _same_start(P, cfg, amps):
    """Two-buffer and AA pipes holding the same state: the log-law start of
    each is the same formula evaluated in a different kernel (results agree
    to an FP32 rounding), so both are given the two-buffer start as exported
    (FP32; for FP64 storage the exported values, written back to both)."""
    ab = P.Pipe(cfg, amps)
    aa = P.Pipe(dict(cfg, pattern=1), amps)
    g_ab, g_aa = _pops(ab), _pops(aa)
    np.testing.assert_allclose(g_aa, g_ab, rtol=2.0 ** -21, atol=1e-12)
    g = torch.from_numpy(g_ab).cuda()
    ab.set_populations(g, step=0)
    aa.set_populations(g, step=0)
    assert np.array_equal(_pops(aa), g_ab) and np.array_equal(_pops(ab), g_ab)
    return ab, aa


@pytest.mark.parametrize("storage", [0, 1, 2])
def test_aa_equals_two_buffer_bitwise(P, storage):
    """Log-law start, six trigger modes: from the same state, populations,
    moments and FP64 diagnostics of the AA run equal the two-buffer run
    after 1, 2, 6, 13 and 23 steps (both parities)."""
    cfg = _cfg(nx=30, ny=28, nz=24, radius=13.4, storage=storage)
    amps = _amps(cfg, seed=9)
    ab, aa = _same_start(P, cfg, amps)
    for n in (1, 1, 4, 7, 10):
        ab.step(n)
        aa.step(n)
        assert aa.step_index == ab.step_index
        assert np.array_equal(_pops(ab), _pops(aa)), f"step {ab.step_index}"
        ra, ua = ab.moments()
        rb, ub = aa.moments()
        assert torch.equal(ra, rb) and torch.equal(ua, ub)
        assert np.array_equal(ab.diagnostics(raise_on_nan=True), aa.diagnostics(raise_on_nan=True))
    _log(f"storage {storage}: AA == two-buffer over {ab.step_index} steps")


@pytest.mark.parametrize("launch", [
    dict(block=64, zchunk=3, xcd_remap=1, pipes_per_launch=2, pipe_major=0),
    dict(block=256, zchunk=1, xcd_remap=0, pipes_per_launch=1, pipe_major=1),
])
def test_aa_batched_graph_and_persistent(P, launch):
    """Three pipes: launch geometries, step order, graph replays at both step
    parities and persistent launches give the two-buffer states."""
    cfg = _cfg(batch=3)
    amps = _amps(cfg, seed=21)
    ab, aa = _same_start(P, cfg, amps)
    aa.set_launch(**launch)
    ab.step(3)
    aa.step(3)
    for n, how in ((10, "graph"), (7, "graph"), (5, "persistent"), (16, "graph"), (6, "persistent")):
        ab.step(n)
        if how == "graph":
            aa.step_graph(n, 4)
        else:
            aa.step_persistent(n)
        assert aa.step_index == ab.step_index
        assert np.array_equal(_pops(ab), _pops(aa)), f"{how} to step {ab.step_index}"


def test_aa_save_load_and_energy(P):
    cfg = _cfg()
    amps = _amps(cfg)
    p = P.Pipe(dict(cfg, pattern=1), amps)
    p.step(5)  # odd: the buffer holds exchanged slots
    blob, s = p.save()
    blob = blob.clone()
    p.step(9)
    a = _pops(p)
    e = p.energy()
    p.load(blob, s)
    assert p.step_index == 5
    p.step(9)
    assert np.array_equal(a, _pops(p))
    ref = P.Pipe(dict(cfg, pattern=1), amps)
    ref.step(14)
    assert np.array_equal(ref.energy(), e)


def test_aa_has_no_recompute(P):
    cfg = _cfg()
    p = P.Pipe(dict(cfg, pattern=1), _amps(cfg))
    ring = torch.empty((2, p.state_bytes), dtype=torch.uint8, device="cuda")
    blob, s = p.save()
    with pytest.raises(P.LbmError):
        p.recompute(blob, s, ring)
