"""The metric workload at its full size (1024^2 cells, 64x64 subdomains of 16^2, 8 elements per
side), run as the bench runs it (FP64, the same kernels), checked where the oracle can follow it:

* identities that hold at any size: MPM-2P with kappa^n = kappa^m returns the conservative
  velocity of the last MRCM update (the perturbation problem of eq:mpm_tf_3 then has zero
  source and data); the downscaled velocity conserves mass in every cell and is the two-point
  flux of a pressure inside every subdomain (its circulation divided by the transmissibilities
  vanishes around every vertex inside a subdomain);
* outputs the oracle computes one by one: the upwind saturation sub-step and the water cut on
  the whole grid, the switch criterion epsilon, and the downscaling problem of sampled
  subdomains given their boundary fluxes.
"""
import math

import numpy as np
import pytest

from oracle import downscale as odown
from oracle import fine, physics, splitting, transport as otrans
from paper_2103_11050_amd import inputs

from .gpu_common import to_np, vel_rel_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def binding():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2103_11050_amd import binding as b
    b.load()
    return b


@pytest.fixture(scope="module")
def workload():
    cfg = inputs.config("c3")
    return cfg, inputs.permeability(cfg), inputs.initial_saturation(cfg)


def _run(binding, cfg, K, s0):
    dev = torch.device("cuda:0")
    return binding.Run(cfg, torch.from_numpy(K).to(dev), torch.from_numpy(s0).to(dev))


def _vel(r):
    ux, uy = r.velocity()
    return to_np(ux), to_np(uy)


def _divergence(cfg, ux, uy):
    ny, nx = ux.shape[0], uy.shape[1]
    hx, hy = cfg["lx"] / nx, cfg["ly"] / ny
    return hy * (ux[:, 1:] - ux[:, :-1]) + hx * (uy[1:, :] - uy[:-1, :])


def _circulation(cfg, kap, ux, uy):
    """Around every vertex inside a subdomain: u/t on the two x-faces and two y-faces of the
    vertex (t the harmonic transmissibility), summed with the signs that cancel the pressures,
    and the scale of its terms."""
    ny, nx = kap.shape
    hx, hy = cfg["lx"] / nx, cfg["ly"] / ny
    tx, ty = fine.interior_trans(kap, hx, hy)
    px = ux[:, 1:-1] / tx          # p_left - p_right, (ny, nx-1)
    py = uy[1:-1, :] / ty          # p_below - p_above, (ny-1, nx)
    circ = px[:-1, :] - px[1:, :] - py[:, :-1] + py[:, 1:]     # vertex (j+1, i+1), (ny-1, nx-1)
    scale = np.abs(px[:-1, :]) + np.abs(px[1:, :]) + np.abs(py[:, :-1]) + np.abs(py[:, 1:])
    mx, my = cfg["sub_x"], cfg["sub_y"]
    # vertex between cells i, i+1 and j, j+1 lies inside a subdomain unless i+1 or j+1 is a
    # multiple of the subdomain size
    inside_x = (np.arange(1, nx) % mx) != 0
    inside_y = (np.arange(1, ny) % my) != 0
    mask = inside_y[:, None] & inside_x[None, :]
    return circ[mask], scale[mask]


def test_mpm_with_unchanged_conductivity_returns_mrcm_velocity(binding, workload):
    """kappa^n = kappa^m: one forced MPM-2P update (local solves, interface solve,
    reconstruction, downscaling at 1024^2) reproduces the MRCM velocity."""
    cfg, K, s0 = workload
    print("[gpu] full size: MPM-2P with unchanged conductivity", flush=True)
    r = _run(binding, cfg, K, s0)
    r.start()
    ux0, uy0 = _vel(r)
    r.velocity_update(binding.FORCE_MPM)
    st = r.stats()
    assert st["error_word"] == 0 and st["last_branch"] == binding.FORCE_MPM
    ux1, uy1 = _vel(r)
    err = vel_rel_err(cfg, ux1, uy1, ux0, uy0)
    print(f"    rel L2 difference {err:.3e}", flush=True)
    assert err <= 1e-10
    r.close()


def test_steps_against_oracle_pieces(binding, workload):
    """Three Algorithm-1 passes at 1024^2; the last one checked piece by piece."""
    cfg, K, s0 = workload
    print("[gpu] full size: three passes", flush=True)
    r = _run(binding, cfg, K, s0)
    r.start()
    for _ in range(2):
        r.step()
    sb = to_np(r.saturation()).copy()
    uxb, uyb = _vel(r)
    stb = r.stats()
    r.step()
    st = r.stats()
    assert st["error_word"] == 0
    assert st["tm"] == 1 and st["last_branch"] == binding.FORCE_MPM     # no new basis in this window
    sa = to_np(r.saturation())
    ux, uy = _vel(r)
    r.close()

    # A9: the upwind sub-step with the velocity and time step of the previous update
    s_ref = otrans.saturation_step(cfg, sb, uxb, uyb, stb["dt"])
    ds = float(np.abs(sa - s_ref).max())
    print(f"    saturation step max abs difference {ds:.3e}", flush=True)
    assert ds <= 1e-12
    assert sa.min() >= -1e-14 and sa.max() <= 1 + 1e-14
    assert math.isclose(st["water_cut"], otrans.water_cut(cfg, sa, uxb, uyb), rel_tol=1e-10, abs_tol=1e-15)
    assert math.isclose(st["dt"], otrans.time_step(cfg, ux, uy), rel_tol=1e-12)

    # A1: epsilon against the conductivity of the only basis (the start)
    kap_n = physics.conductivity(sa, K, cfg["mu_w"], cfg["mu_o"])
    kap_m = physics.conductivity(s0, K, cfg["mu_w"], cfg["mu_o"])
    eps = splitting.eps_norm(cfg, kap_n, kap_m)
    assert math.isclose(st["eps"], eps, rel_tol=1e-9), (st["eps"], eps)

    # A8 (every cell): conservation; inside every subdomain a two-point flux of kappa^n
    div = _divergence(cfg, ux, uy)
    hx = cfg["lx"] / cfg["nx"]
    umax = max(float(np.abs(ux).max()), float(np.abs(uy).max()))
    assert float(np.abs(div).max()) <= 1e-11 * umax * hx
    circ, scale = _circulation(cfg, kap_n, ux, uy)
    rel = float((np.abs(circ) / np.maximum(scale, 1e-300)).max())
    print(f"    largest relative circulation inside subdomains {rel:.3e}", flush=True)
    assert rel <= 1e-9

    # A8 (sampled subdomains): the oracle's downscaling given the boundary fluxes
    mx, my = cfg["sub_x"], cfg["sub_y"]
    Sx, Sy = cfg["nx"] // mx, cfg["ny"] // my
    hy = cfg["ly"] / cfg["ny"]
    for I, J in [(0, 0), (Sx - 1, Sy - 1), (0, Sy // 2), (Sx // 2, 0), (17, 42), (Sx - 1, 5)]:
        j0, i0 = J * my, I * mx
        win = dict(cfg, nx=mx, ny=my, lx=mx * hx, ly=my * hy, ne_x=1, ne_y=1)
        uxw = ux[j0:j0 + my, i0:i0 + mx + 1].copy()
        uyw = uy[j0:j0 + my + 1, i0:i0 + mx].copy()
        rx, ry, _ = odown.downscale(win, kap_n[j0:j0 + my, i0:i0 + mx], uxw, uyw)
        scale_w = max(float(np.abs(uxw).max()), float(np.abs(uyw).max()))
        d = max(float(np.abs(rx - uxw).max()), float(np.abs(ry - uyw).max()))
        assert d <= 1e-9 * scale_w, (I, J, d, scale_w)
