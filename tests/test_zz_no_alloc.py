"""The allocation-free entry point (mpm_create_static): a run whose workspace is the library's own
device array gives the same velocities, saturations and counters as a run on a caller-allocated
workspace (mpm_create), on two runs in a row, the second on a smaller grid (the array then holds
the first run's contents), and refuses a second live run on the device and a batch."""
import ctypes

import numpy as np
import pytest

from paper_2103_11050_amd import inputs

from .gpu_common import FP64_FACE_TOL, FP64_SAT_TOL, FP64_VEL_TOL, sat_rel_err, to_np, vel_face_err, vel_rel_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def binding():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2103_11050_amd import binding as b
    b.load()
    return b


def _run_pair(binding, cfg, passes):
    K = inputs.permeability(cfg)
    s0 = inputs.initial_saturation(cfg)
    dev = torch.device("cuda:0")
    Kd, sd = torch.from_numpy(K).to(dev), torch.from_numpy(s0).to(dev)
    out = []
    for static in (False, True):
        r = binding.Run(cfg, Kd, sd, static=static)
        r.start()
        for k in range(passes):
            r.step(binding.FORCE_MRCM if k == passes // 2 else binding.AUTO)
        ux, uy = r.velocity()
        s = r.saturation()
        st = r.stats()
        out.append((to_np(ux).copy(), to_np(uy).copy(), to_np(s).copy(), st))
        r.close()
    return out


@pytest.mark.parametrize("name, kw, passes", [
    ("c2", dict(), 6),                    # 256^2: 49.8 MiB of the 64 MiB array
    ("c1", dict(), 8),                    # then a smaller grid in the same array
])
def test_static_workspace_equals_caller_workspace(binding, name, kw, passes):
    cfg = inputs.config(name, **kw)
    need = binding.workspace_size(cfg)
    print(f"[gpu] static workspace: {name} {cfg['nx']}x{cfg['ny']} ({need / 2**20:.1f} MiB), {passes} passes",
          flush=True)
    (ux0, uy0, s0, st0), (ux1, uy1, s1, st1) = _run_pair(binding, cfg, passes)
    assert st0["error_word"] == 0 and st1["error_word"] == 0
    for key in ("te", "tm", "n_transport", "last_branch", "breakthrough"):
        assert st0[key] == st1[key], key
    for key in ("eps", "t", "pvi", "water_cut", "dt"):
        assert st1[key] == pytest.approx(st0[key], rel=1e-12, abs=1e-300), key
    ev = vel_rel_err(cfg, ux1, uy1, ux0, uy0)
    ef = vel_face_err(ux1, uy1, ux0, uy0)
    es = sat_rel_err(s1, s0)
    print(f"    velocity rel L2 {ev:.2e}, face {ef:.2e}, saturation rel L1 {es:.2e}", flush=True)
    assert ev <= FP64_VEL_TOL and ef <= FP64_FACE_TOL and es <= FP64_SAT_TOL


def test_static_workspace_is_exclusive_and_not_batched(binding):
    cfg = inputs.config("c1")
    dev = torch.device("cuda:0")
    K = torch.from_numpy(inputs.permeability(cfg)).to(dev)
    s0 = torch.from_numpy(inputs.initial_saturation(cfg)).to(dev)
    r = binding.Run(cfg, K, s0, static=True)
    try:
        with pytest.raises(binding.MpmError) as e:
            binding.Run(cfg, K, s0, static=True)
        assert e.value.status == binding.MPM_ESTATE
        b = binding.Batch(2)
        assert binding.load().mpm_batch_attach(b.h, 0, r.h) == binding.MPM_ESTATE
        b.close()
        r.start()
        r.step()
        assert r.stats()["error_word"] == 0
    finally:
        r.close()
    # released by mpm_destroy: the device's array can be taken again
    r2 = binding.Run(cfg, K, s0, static=True)
    r2.close()


def test_static_workspace_refuses_large_runs(binding):
    cfg = inputs.config("c2", nx=512, ny=512)
    d = binding.make_desc(cfg)
    h = ctypes.c_void_p()
    lib = binding.load()
    assert lib.mpm_create_static(ctypes.byref(d), None, ctypes.byref(h)) == binding.MPM_ENOMEM
    assert not h.value
    buf = ctypes.create_string_buffer(256)
    lib.mpm_last_error(None, buf, 256)
    assert b"static array" in buf.value
