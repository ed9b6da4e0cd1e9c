"""The stored oracle values of the metric workload (tests/golden/c3_reference.py) against what
the method fixes without rerunning the oracle (CPU): every stored velocity tile conserves mass in
each cell (q = 0; eq. mpm_upd and the MRCM downscaling are conservative), the saturation stays in
[0, 1], PVI equals the time for unit inflow on a unit square, the velocity norm is consistent
with its projections, and the projection estimator behaves as its chi-square law says on a
known vector."""
import numpy as np
import pytest

from paper_2103_11050_amd import inputs

from .golden import c3_reference as ref_mod


@pytest.fixture(scope="module")
def ref():
    return ref_mod.load()


def test_tiles_conserve_mass(ref):
    cfg = inputs.config("c3")
    hx, hy = cfg["lx"] / cfg["nx"], cfg["ly"] / cfg["ny"]
    for p in range(len(ref["branches"])):
        ux, uy = ref["ux"][p], ref["uy"][p]
        div = hy * (ux[:, :, 1:] - ux[:, :, :-1]) + hx * (uy[:, 1:, :] - uy[:, :-1, :])
        # (each cell holds its share of the subdomain's compatibility defect, the rounding of the
        # 129,024-unknown interface solve spread over 256 cells: about 1e-13 of a face flux)
        assert float(np.abs(div).max()) <= 1e-12 * float(ref["umax"][p]) * hx, p


def test_scalars(ref):
    assert list(ref["branches"]) == ["start", "mpm", "mpm", "mrcm"]
    s = ref["s"]
    assert s.min() >= -1e-12 and s.max() <= 1 + 1e-12
    assert np.all(s[0] == 0.0)                     # s^0 = 0 before any transport
    np.testing.assert_allclose(ref["pvi"], ref["t"], rtol=1e-12, atol=0)
    assert np.all(np.diff(ref["t"]) > 0)
    assert ref["eps"][0] == inputs.config("c3")["eta"] and ref["eps"][3] == 0.0   # eps = eta; new basis
    assert np.all(ref["eps"][1:3] > 0)


def test_projection_norm_estimate(ref):
    """The stored projections estimate the stored norms (chi-square with 256 degrees of freedom:
    within a factor 0.7 to 1.3 except with probability 3.3e-11), and the estimator is linear."""
    for p in range(len(ref["branches"])):
        est = float(np.linalg.norm(ref["uproj"][p])) / float(ref["unorm"][p])
        assert 0.7 <= est <= 1.3, (p, est)
    v = np.random.default_rng(1).standard_normal(1000)
    w = np.random.default_rng(2).standard_normal(1000)
    pv, pw, pvw = ref_mod.projections(v, w, 2 * v - w)
    np.testing.assert_allclose(pvw, 2 * pv - pw, rtol=1e-12, atol=1e-12)
    assert 0.7 <= np.linalg.norm(pv) / np.linalg.norm(v) <= 1.3
