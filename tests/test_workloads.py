"""The seeded input generators: determinism, shapes, band limits, ranges."""
import numpy as np

from paper_2403_06654_amd import workloads as W


def test_deterministic_and_shapes():
    a = W.c1_inputs(seed=3)
    b = W.c1_inputs(seed=3)
    np.testing.assert_array_equal(a["f"], b["f"])
    assert a["rho"].shape == (256,) and a["f"].shape == (256,)
    assert not np.array_equal(W.c1_inputs(seed=4)["f"], a["f"])


def test_band_limit_and_mean():
    u = W.band_limited((32, 16, 64), 8, seed=1)
    uh = np.fft.rfftn(u)
    assert abs(uh[0, 0, 0]) < 1e-9 * np.abs(uh).max()
    kz = np.abs(np.fft.fftfreq(32, 1 / 32))[:, None, None]
    ky = np.abs(np.fft.fftfreq(16, 1 / 16))[None, :, None]
    kx = np.arange(33)[None, None, :]
    out = (kz > 8) | (ky > 8) | (kx > 8)
    assert np.abs(uh[np.broadcast_to(out, uh.shape)]).max() < 1e-9 * np.abs(uh).max()
    assert abs(np.sqrt(np.mean(u * u)) - 1) < 1e-12
    g = W.band_limited((16, 16), 4, seed=1, keep_mean=True)
    assert abs(g.mean()) > 1e-6


def test_density_ranges():
    rho = W.tophat_1d(256)
    assert rho.min() > 0.99 and rho.max() < 3.01 and rho.max() > 2.99
    j = W.jet_density(32, 5.0)
    assert j.shape == (32, 32, 32) and j.min() > 0.99 and j.max() <= 5.0 + 1e-12
    j = W.jet_density(32, 0.5)
    assert j.min() >= 0.5 - 1e-12 and j.max() < 1.01
    s = W.slab_density_2d(64, 7.0, seed=2)
    assert s.min() > 0.99 and s.max() < 7.01
    reqs = W.serving_requests(64)
    assert {r["n"] for r in reqs} <= {128, 256, 512, 1024}
    assert all(1.5 <= r["r"] <= 10 for r in reqs)
    c2 = W.c2_inputs(nx=32, m=16)
    assert c2["rho"].shape == (17, 32) and c2["f"].shape == (17, 32)
    assert c2["rho"].min() > 0.99 and c2["rho"].max() < 3.01
    c5 = W.c5_density(32)
    assert c5.min() > 0.99 and c5.max() < 10.01
