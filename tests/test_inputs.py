"""Seeded input generators (CPU): the self-similar field of the Section 5.1 experiment and the
batched and served workload lists."""
import numpy as np

from paper_2103_11050_amd import inputs


def test_self_similar_field_spectrum_and_scale():
    """Power spectrum |k|^(beta - 2) = |k|^-1.5 for the covariance |x - y|^-1/2 (its 2-D Fourier
    transform), zero mean, unit range, reproducible from the seed."""
    f = inputs.self_similar_field(256, 256, 1.0, 1.0, seed=3)
    assert abs(f.mean()) < 1e-12 and abs((f.max() - f.min()) - 1.0) < 1e-12
    assert np.array_equal(f, inputs.self_similar_field(256, 256, 1.0, 1.0, seed=3))
    slopes = []
    for seed in range(4):
        g = inputs.self_similar_field(256, 256, 1.0, 1.0, seed=seed)
        P = np.abs(np.fft.fft2(g)) ** 2
        k = np.sqrt(np.fft.fftfreq(256)[:, None] ** 2 + np.fft.fftfreq(256)[None, :] ** 2)
        m = (k > 0.02) & (k < 0.3)
        slopes.append(np.polyfit(np.log(k[m]), np.log(P[m]), 1)[0])
    assert abs(np.mean(slopes) + 1.5) < 0.08, slopes


def test_x1_permeability_contrast():
    for contrast in (1e3, 1e6):
        cfg = inputs.x1_config(contrast)
        K = inputs.permeability(cfg)
        assert K.shape == (64, 64)
        assert abs(K.max() / K.min() / contrast - 1.0) < 1e-9
        # K = 0.8 exp(delta xi) with xi of zero mean: the geometric mean is 0.8
        assert abs(np.exp(np.log(K).mean()) - 0.8) < 1e-12
    cfg = inputs.x1_config(ne=2, cn=20)
    assert cfg["bc_kind"][:2] == [inputs.PRESSURE, inputs.PRESSURE] and cfg["bc_value"][:2] == [1.0, 0.0]
    assert cfg["ne_x"] == 2 and cfg["cn"] == 20 and cfg["mu_o"] == 40.0 and cfg["eta"] == 1e-2


def test_batch_and_serve_workloads():
    b = inputs.batch_workload(9)
    assert [(c["nx"], c["sub_x"]) for c in b[:3]] == [(64, 8), (128, 16), (256, 32)]
    assert [c["seed"] for c in b] == list(range(1000, 1009))
    r = inputs.serve_requests(64)
    assert {c["nx"] for c in r} <= {128, 256, 512}
    assert all(10.0 <= c["mu_o"] <= 100.0 and 1.0 <= c["sigma2"] <= 4.0 for c in r)
    assert r[0] == inputs.serve_requests(64)[0]


def test_x4_finger_growth_workload():
    """300 x 50 cells on [0,3] x [0,1/2] in 20 x 10 subdomains with one fine face per element,
    M = 4, homogeneous K, p = 0 / -1e4, and a water front advanced at the channel centre."""
    cfg = inputs.x4_config()
    assert (cfg["nx"], cfg["ny"], cfg["sub_x"], cfg["sub_y"]) == (300, 50, 20, 10)
    assert (cfg["ne_x"], cfg["ne_y"]) == (20, 10) and cfg["mu_o"] / cfg["mu_w"] == 4.0
    assert cfg["bc_value"][:2] == [0.0, -1.0e4]
    K = inputs.permeability(cfg)
    assert K.shape == (50, 300) and np.all(K == 1.0)
    s = inputs.initial_saturation(cfg)
    assert set(np.unique(s)) == {0.0, 1.0}
    front = s.sum(axis=1)                 # saturated cells per row
    assert front[0] == front[-1] == 10 and front[25] == 15
    assert front.max() == 15 and np.all(front[np.abs(np.arange(50) + 0.5 - 25) >= 5] == 10)


def test_x1_basis_count_matches_cost_model():
    """The experiment's N-hat (RCR of Section 4.3) agrees with the cost model for constant and
    linear interface spaces."""
    from oracle import cost
    from paper_2103_11050_amd import x1
    for ne in (1, 2):
        for deg in (0, 1):
            cfg = dict(inputs.x1_config(1e3, ne=ne, cn=1), iface_degree=deg)
            sx, sy = cfg["nx"] // cfg["sub_x"], cfg["ny"] // cfg["sub_y"]
            assert x1.homogeneous_bf_count(cfg) == cost.homogeneous_bf_count(sx, sy, ne, ne, kU=deg + 1, kP=deg + 1)
