"""Batched ensembles on the GPU: launch geometry, step order, graph replay and
the autotuner leave the results bitwise unchanged (needs an MI355X)."""
import os
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


def _cfg(batch=5):
    cfg = LI.preset("batched")
    cfg.update(nx=22, ny=22, nz=20, radius=10.4, batch=batch)
    cfg["period"] = float(round(0.052 * 10.4 / cfg["u_tau"]))
    return cfg


def _amps(cfg):
    return LI.preset_amplitudes(cfg) * 5.0


@pytest.mark.parametrize("launch", [
    dict(block=64, zchunk=3, xcd_remap=1, pipes_per_launch=2, pipe_major=0),
    dict(block=128, zchunk=20, xcd_remap=0, pipes_per_launch=1, pipe_major=1),
    dict(block=256, zchunk=1, xcd_remap=1, pipes_per_launch=3, pipe_major=1),
    dict(block=512, zchunk=2, xcd_remap=8, pipes_per_launch=5, pipe_major=0),
])
def test_launch_geometry_and_order_do_not_change_results(P, launch):
    cfg = _cfg()
    amps = _amps(cfg)
    ref = P.Pipe(cfg, amps)
    ref.step(23)
    gref = ref.populations().cpu().numpy()
    p = P.Pipe(cfg, amps)
    p.set_launch(**launch)
    p.step(11)
    p.step_graph(12, 4)
    assert p.step_index == 23
    assert np.array_equal(p.populations().cpu().numpy(), gref)


def test_autotune_restores_state_and_caches(P, tmp_path):
    from paper_2405_12082_amd import autotune
    cfg = _cfg(batch=4)
    amps = _amps(cfg)
    p = P.Pipe(cfg, amps)
    p.step(5)
    before = p.populations().cpu().numpy()
    cache = os.path.join(tmp_path, "tune.json")
    r = autotune.autotune(p, steps=3, cache_path=cache)
    _log(f"autotune best {r['best']} {r['ms_per_step']:.4f} ms/step over {r['tried']} candidates")
    assert not r["cached"] and r["tried"] > 50
    assert p.step_index == 5
    assert np.array_equal(p.populations().cpu().numpy(), before)
    r2 = autotune.autotune(P.Pipe(cfg, amps), cache_path=cache)
    assert r2["cached"] and r2["best"] == r["best"]
    # the tuned geometry gives the same trajectory
    p.step(9)
    q = P.Pipe(cfg, amps)
    q.step(14)
    assert np.array_equal(p.populations().cpu().numpy(), q.populations().cpu().numpy())


def test_set_launch_rejects_bad_values(P):
    p = P.Pipe(_cfg(batch=2), _amps(_cfg(batch=2)))
    for bad in (dict(block=1024), dict(zchunk=65), dict(xcd_remap=4097), dict(pipes_per_launch=3),
                dict(pipe_major=2)):
        with pytest.raises(P.LbmError):
            p.set_launch(**bad)


@pytest.mark.parametrize("block,zchunk", [(256, 1), (64, 4), (512, 1)])
def test_persistent_launch_equals_eager(P, block, zchunk):
    """One cooperative launch of n steps with a grid barrier between steps
    gives the same states as n ordinary launches (both buffer parities)."""
    cfg = _cfg(batch=3)
    amps = _amps(cfg)
    ref = P.Pipe(cfg, amps)
    p = P.Pipe(cfg, amps)
    p.set_launch(block=block, zchunk=zchunk)
    for n in (1, 13, 6):
        ref.step(n)
        p.step_persistent(n)
        assert p.step_index == ref.step_index
        assert np.array_equal(p.populations().cpu().numpy(), ref.populations().cpu().numpy()), n


@pytest.mark.parametrize("pattern,wall,k", [(0, 0, 4), (1, 0, 6), (0, 1, 4)])
def test_persistent_graph_equals_eager(P, pattern, wall, k):
    """Replays of a graph holding one persistent launch of k steps (three
    pipes; two buffers, AA and the interpolated wall): the states of n
    ordinary launches after every call, including a remainder of n mod k
    steps, a second replay of the cached graph and a call after a change of
    the launch geometry (which recaptures it)."""
    cfg = dict(_cfg(batch=3), pattern=pattern, wall=wall)
    amps = _amps(cfg)
    ref = P.Pipe(cfg, amps)
    p = P.Pipe(cfg, amps)
    _log(f"persistent graph pattern={pattern} wall={wall} k={k}")
    for n in (3, 2 * k + 2, k, 1):
        ref.step(n)
        p.step_persistent_graph(n, k)
        assert p.step_index == ref.step_index
        assert np.array_equal(p.populations().cpu().numpy(), ref.populations().cpu().numpy()), n
    p.set_launch(block=64, zchunk=2)
    ref.step(2 * k)
    p.step_persistent_graph(2 * k, k)
    assert np.array_equal(p.populations().cpu().numpy(), ref.populations().cpu().numpy())
    with pytest.raises(P.LbmError):
        p.step_persistent_graph(4, 3)


def test_choose_pattern_tunes_both_patterns(P, tmp_path):
    from paper_2405_12082_amd import autotune
    cfg = _cfg(batch=2)
    amps = _amps(cfg)
    cache = os.path.join(tmp_path, "tune.json")
    r = autotune.choose_pattern(cfg, amps, steps=2, cache_path=cache)
    _log(f"choose_pattern: {r}")
    assert r["pattern"] in (0, 1) and set(r["by_pattern"]) == {0, 1} and not r["cached"]
    assert r["ms_per_step"] == min(r["by_pattern"].values())
    r2 = autotune.choose_pattern(cfg, amps, cache_path=cache)
    assert r2["cached"] and r2["pattern"] == r["pattern"] and r2["best"] == r["best"]
    # the adjoint needs two buffers
    r3 = autotune.choose_pattern(dict(cfg, adjoint=1), amps, steps=2, cache_path=cache)
    assert r3["pattern"] == 0 and set(r3["by_pattern"]) == {0}


def test_full_size_ensemble_in_the_bench_launch(P):
    """The 64-pipe ensemble (64 x 64 x 256, R = 30, own seeded forcing each)
    in the launch the autotuner picks for the bench: AA in place, 128
    threads, 3 pipes per launch in pipe-major order, XCD eighths, replays of
    a 50-step graph.  After 100 steps, density and velocity of pipes 0, 31
    and 63 equal independent single-pipe runs (two buffers, default launch)
    bitwise."""
    cfg = LI.preset("batched")
    amps = LI.preset_amplitudes(cfg)
    ens = P.Pipe(dict(cfg, pattern=1), amps)
    ens.set_launch(block=128, zchunk=1, xcd_remap=1, pipes_per_launch=3, pipe_major=1)
    ens.step_graph(100, 50)
    rho, u = ens.moments()
    for b in (0, 31, 63):
        one = P.Pipe(dict(cfg, batch=1), amps[b:b + 1])
        one.step(100)
        r1, u1 = one.moments()
        assert torch.equal(rho[b], r1[0]) and torch.equal(u[b], u1[0]), b
        del one
    assert (ens.diagnostics()[:, 4] == 0).all()


@pytest.mark.parametrize("mode", ["graph_aa", "graph_ab", "persistent_graph_aa", "persistent_graph_ab"])
def test_batched_pipes_each_match_their_oracle(P, oracle_mod, mode):
    """Three pipes with distinct seeded forcing and distinct random states,
    two steps through the ensemble launches (AA or two buffers, one pipe per
    launch in pipe-major order with XCD eighths as the bench's tuned
    ensemble, as graph replay or as one persistent launch in a graph): each
    pipe equals its own oracle pipe within the tolerance of two single steps,
    128 * 2^-24 * (max|g_in| + max|g_out|)."""
    O = oracle_mod
    pattern = 1 if mode.endswith("_aa") else 0
    cfg = dict(nx=21, ny=23, nz=13, batch=3, radius=9.6, tau=0.56, accel_z=3e-6, n_modes=6, kz=3.0,
               kappa=0.5, l0_frac=0.2, l_frac=0.4, period=40.0, force_off_step=1000, storage=0, wall=0,
               pattern=pattern, init=1, u_tau=0.01)
    amps = LI.batch_amplitudes(17, 3, 6, cfg["u_tau"], cfg["period"]) * 40.0
    o1 = O.Pipe(O.make_config(**cfg), amps[0])
    mask = o1.fluid_mask()
    _, w, _ = O.lattice()
    g0 = np.stack([LI.random_deviations(300 + b, (cfg["nz"], cfg["ny"], cfg["nx"])) for b in range(3)])
    g0[:, :, ~mask] = 0.0
    p = P.Pipe(cfg, amps)
    p.set_launch(block=128, zchunk=1, xcd_remap=1, pipes_per_launch=1, pipe_major=1)
    p.set_populations(torch.from_numpy(g0).cuda(), step=10)
    _log(f"batched vs oracle: {mode}")
    if mode.startswith("graph"):
        p.step_graph(2, 2)
    else:
        p.step_persistent_graph(2, 2)
    g2 = p.populations().cpu().numpy().astype(np.float64)
    for b in range(3):
        o = O.Pipe(O.make_config(**cfg), amps[b])
        f0 = g0[b].astype(np.float64) + w[:, None, None, None]
        f0[:, ~mask] = 0.0
        o.set_f(f0, 10)
        o.step(2)
        go = o.get_f() - w[:, None, None, None]
        err = np.abs(g2[b][:, mask] - go[:, mask]).max()
        tol = 128 * 2.0 ** -24 * (np.abs(g0[b]).max() + np.abs(go[:, mask]).max())
        _log(f"  pipe {b}: error {err:.3e} (tolerance {tol:.3e})")
        assert err <= tol, b
