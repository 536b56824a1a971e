"""The allocation-free, context-free spectrum entry point
(lbm_ring_spectrum_static, its twiddles in a library-owned device array)
against the context's lbm_ring_spectrum on the same ring samples, through
the C-ABI (needs an MI355X).  Two calls in a row, the second smaller (fewer
pipes, planes and ring points): the scratch keeps the first call's table,
so the second call must rewrite what it uses.  Spectra and plane averages
agree to FP64 rounding (the twiddles come from the device's sincospi
instead of the host's cos/sin: within 1e-12 of the largest value), the
dominant modes exactly."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2405_12082_amd as P
    P.lib()
    return P


def _rings(seed, batch, nz, ntheta, modes):
    """Seeded ring samples: a few azimuthal modes per pipe plus noise."""
    rng = np.random.default_rng(seed)
    th = 2 * np.pi * np.arange(ntheta) / ntheta
    r = 0.05 + 1e-3 * rng.standard_normal((batch, nz, ntheta))
    for b in range(batch):
        for m, a in modes[b]:
            r[b] += a * np.cos(m * th + rng.uniform(0, 2 * np.pi, size=(nz, 1)))
    return torch.from_numpy(r.astype(np.float32)).cuda()


def _static(P, ring, mmax, stream):
    B, nz, n = ring.shape
    spec = torch.full((B, nz, mmax + 1), np.nan, dtype=torch.float64, device="cuda")
    mean = torch.full((B, mmax + 1), np.nan, dtype=torch.float64, device="cuda")
    dom = torch.full((B,), -1, dtype=torch.int32, device="cuda")
    rc = P.lib().lbm_ring_spectrum_static(C.c_void_p(ring.data_ptr()), B, nz, n, mmax, C.c_void_p(spec.data_ptr()),
                                          C.c_void_p(mean.data_ptr()), C.c_void_p(dom.data_ptr()),
                                          C.c_void_p(stream.cuda_stream))
    assert rc == 0
    return spec, mean, dom


def _context(P, ring, mmax, stream):
    B, nz, n = ring.shape
    p = P.Pipe(dict(nx=12, ny=12, nz=nz, batch=B, radius=5.0, tau=0.8), stream=stream)
    out = p.ring_spectrum(ring, mmax)
    torch.cuda.synchronize()
    p.close()
    return out


def _compare(a, b):
    sa, ma, da = (t.cpu().numpy() for t in a)
    sb, mb, db = (t.cpu().numpy() for t in b)
    assert np.isfinite(sa).all() and np.isfinite(ma).all()
    assert np.abs(sa - sb).max() <= 1e-12 * np.abs(sb).max()
    assert np.abs(ma - mb).max() <= 1e-12 * np.abs(mb).max()
    assert np.array_equal(da, db)
    return da


def test_static_spectrum_equals_context_spectrum_twice(P):
    stream = torch.cuda.current_stream()
    # first call: 3 pipes x 40 planes x 1024 points (the static call comes
    # first, so in a fresh process it also sets up the scratch address)
    r1 = _rings(1, 3, 40, 1024, [[(5, 0.02)], [(3, 0.01), (7, 0.02)], [(2, 0.03)]])
    s1 = _static(P, r1, 10, stream)
    torch.cuda.synchronize()
    d1 = _compare(s1, _context(P, r1, 10, stream))
    assert list(d1) == [5, 7, 2]
    # second call, smaller: 1 pipe x 7 planes x 256 points, fewer modes
    r2 = _rings(2, 1, 7, 256, [[(4, 0.02), (6, 0.005)]])
    s2 = _static(P, r2, 6, stream)
    torch.cuda.synchronize()
    d2 = _compare(s2, _context(P, r2, 6, stream))
    assert list(d2) == [4]


def test_static_spectrum_rejects_bad_arguments(P):
    stream = torch.cuda.current_stream()
    ring = torch.zeros((1, 2, 64), dtype=torch.float32, device="cuda")
    spec = torch.zeros((1, 2, 5), dtype=torch.float64, device="cuda")
    mean = torch.zeros((1, 5), dtype=torch.float64, device="cuda")
    dom = torch.zeros((1,), dtype=torch.int32, device="cuda")
    L = P.lib()
    vp = lambda t: C.c_void_p(t.data_ptr())
    s = C.c_void_p(stream.cuda_stream)
    for args in ((None, 1, 2, 64, 4, vp(spec), vp(mean), vp(dom)),      # no ring
                 (vp(ring), 0, 2, 64, 4, vp(spec), vp(mean), vp(dom)),  # batch < 1
                 (vp(ring), 1, 2, 4097, 4, vp(spec), vp(mean), vp(dom)),  # beyond the scratch
                 (vp(ring), 1, 2, 64, 33, vp(spec), vp(mean), vp(dom)),  # mmax > ntheta / 2
                 (vp(ring), 1, 2, 64, 4, vp(spec), None, vp(dom))):     # dominant without mean
        assert L.lbm_ring_spectrum_static(*args, s) == P._lib.LBM_EINVAL
