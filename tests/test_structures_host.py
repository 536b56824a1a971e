"""The package's mode-series statistics (host code, no GPU) against the
oracle's loop versions on random and Markov series: equal to rounding."""
import numpy as np

from oracle import structures as S
from paper_2405_12082_amd import structures as H


def _series(seed, n=3000, k=10):
    rng = np.random.default_rng(seed)
    T = np.eye(k) * 0.9 + 0.1 / k
    s, out = 1, []
    for _ in range(n):
        out.append(s + 1)
        s = rng.choice(k, p=T[:, s])
    return out


def test_transition_matrix_matches_oracle():
    for seed in (1, 2):
        modes = _series(seed)
        for lag in (1, 3):
            np.testing.assert_allclose(H.transition_matrix(modes, 10, lag), S.transition_matrix(modes, lag, 10),
                                       rtol=0, atol=1e-15)


def test_ck_test_matches_oracle():
    modes = _series(3)
    ours = H.ck_test(modes, 10, (1, 2, 5))
    ref = S.ck_eigenvalues(modes, 10, (1, 2, 5))
    for (d, lam, pred), (lam_o, pred_o) in zip(ours, ref):
        np.testing.assert_allclose(lam, lam_o, atol=1e-12)
        np.testing.assert_allclose(pred, pred_o, atol=1e-12)


def test_self_correlation_matches_oracle():
    modes = _series(4, n=800)
    f, mean = H.self_correlation(modes, 10, 30)
    fo, mo = S.self_correlation(modes, 10, 30)
    np.testing.assert_allclose(f, fo, atol=1e-12)
    np.testing.assert_allclose(mean, mo, atol=1e-12)


def test_streamwise_lengths_match_oracle_runs():
    modes = _series(5, n=2000)
    lengths = H.streamwise_lengths(modes, 10, dt_steps=20, u_conv=0.05)
    runs = S.run_lengths(modes, 10)
    for k in range(1, 11):
        r = np.array(runs[k], float) * 20 * 0.05
        assert lengths[k] == ((r.mean(), r.max()) if r.size else (0.0, 0.0))
