"""Batched and served forms (GPU only): runs of different sizes stepped together in one batch,
each on its own stream, give bitwise the results of the same runs stepped alone; slots can be
emptied and refilled between steps; breakthrough stops a run."""
import numpy as np
import pytest

from paper_2103_11050_amd import inputs

from .gpu_common import to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def binding():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2103_11050_amd import binding as b
    b.load()
    return b


PROBLEMS = [
    # seed, nx, ny, sub, ne, overrides
    (101, 32, 32, 8, 2, dict(sigma2=2.0, corr_len=0.2, mu_o=20.0, eta=0.01)),
    (102, 64, 48, 16, 4, dict(sigma2=3.0, corr_len=0.1, mu_o=50.0, eta=0.05)),
    (103, 48, 48, 8, 4, dict(sigma2=1.0, corr_len=0.2, mu_o=10.0, eta=0.02, switch_rule="text")),
    (104, 64, 64, 16, 8, dict(sigma2=4.0, corr_len=0.1, mu_o=100.0, eta=0.1)),
]


def _make(binding, p, stream=None):
    seed, nx, ny, sub, ne, kw = p
    cfg, K = inputs.random_problem(seed, nx, ny, sub, sub, ne, ne, **kw)
    dev = torch.device("cuda:0")
    Kt = torch.from_numpy(np.ascontiguousarray(K)).to(dev)
    st = torch.from_numpy(np.ascontiguousarray(inputs.initial_saturation(cfg))).to(dev)
    torch.cuda.synchronize()
    r = binding.Run(cfg, Kt, st, stream=stream)
    r.start()
    return r


def _state(r):
    torch.cuda.synchronize()
    ux, uy = r.velocity()
    s = r.saturation()
    st = r.stats()
    torch.cuda.synchronize()
    return to_np(ux), to_np(uy), to_np(s), st


def _same(a, b):
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
    for k in ("te", "tm", "eps", "pvi", "water_cut", "last_branch"):
        assert a[3][k] == b[3][k], (k, a[3][k], b[3][k])


def test_batch_equals_solo(binding):
    nsteps = 12
    print("[gpu] batch of", len(PROBLEMS), "runs,", nsteps, "steps", flush=True)
    solo = []
    for p in PROBLEMS:
        r = _make(binding, p)
        for _ in range(nsteps):
            r.step()
        solo.append(_state(r))
        r.close()
    streams = [torch.cuda.Stream() for _ in PROBLEMS]
    runs = [_make(binding, p, s) for p, s in zip(PROBLEMS, streams)]
    b = binding.Batch(len(runs) + 1)          # one slot left empty
    for i, r in enumerate(runs):
        b.attach(i, r)
    for _ in range(nsteps):
        b.step()
    for r, ref in zip(runs, solo):
        _same(_state(r), ref)
    assert any(ref[3]["tm"] > 1 for ref in solo), "no basis update exercised"
    b.close()
    for r in runs:
        r.close()


def test_slots_refilled_between_steps(binding):
    """Continuous batching: a run leaves its slot for some steps (its state is untouched), a new
    run takes another slot mid-way, and every run ends equal to its solo run with the same
    number of steps."""
    p0, p1, p2 = PROBLEMS[0], PROBLEMS[1], PROBLEMS[3]
    streams = [torch.cuda.Stream() for _ in range(3)]
    r0, r1 = _make(binding, p0, streams[0]), _make(binding, p1, streams[1])
    b = binding.Batch(2)
    b.attach(0, r0)
    b.attach(1, r1)
    n0 = n1 = n2 = 0
    for _ in range(3):
        b.step()
        n0 += 1
        n1 += 1
    b.detach(0)                       # r0 waits
    for _ in range(2):
        b.step()
        n1 += 1
    r2 = _make(binding, p2, streams[2])
    b.attach(0, r2)                   # a new request takes the freed slot
    for _ in range(4):
        b.step()
        n1 += 1
        n2 += 1
    b.step([False, True])             # only slot 1
    n1 += 1
    b.detach(1)
    b.attach(1, r0)                   # r0 comes back
    for _ in range(2):
        b.step()
        n0 += 1
        n2 += 1
    got = {0: _state(r0), 1: _state(r1), 2: _state(r2)}
    for key, p, n in ((0, p0, n0), (1, p1, n1), (2, p2, n2)):
        r = _make(binding, p)
        for _ in range(n):
            r.step()
        _same(got[key], _state(r))
        r.close()
    b.close()
    for r in (r0, r1, r2):
        r.close()


def test_advance_stops_at_breakthrough(binding):
    cfg, K = inputs.random_problem(7, 32, 16, 8, 8, 2, 2, sigma2=1.0, corr_len=0.3, mu_o=5.0, eta=0.05)
    dev = torch.device("cuda:0")
    Kt = torch.from_numpy(np.ascontiguousarray(K)).to(dev)
    st = torch.from_numpy(np.zeros_like(K)).to(dev)
    r = binding.Run(cfg, Kt, st)
    r.start()
    done = r.advance(5000, True)
    s = r.stats()
    assert s["breakthrough"] == 1 and s["water_cut"] >= cfg["breakthrough_cut"]
    assert s["te"] == done + 1
    # stepping one by one gives the same first breakthrough step
    r2 = binding.Run(cfg, Kt, st)
    r2.start()
    n = 0
    while True:
        r2.step()
        n += 1
        if r2.stats()["breakthrough"]:
            break
    assert n == done
    _same(_state(r), _state(r2))
    r.close()
    r2.close()


def test_served_equals_alone(binding):
    """Requests admitted over time into the batch (fewer slots than requests, so some wait)
    finish with bitwise the results of the same runs advanced alone to breakthrough."""
    from paper_2103_11050_amd import serve
    reqs = inputs.serve_requests(5, grids=(32, 64))
    for c in reqs:
        c.update(sub_x=8, sub_y=8, ne_x=2, ne_y=2)
    arrivals = [0.0, 0.0, 0.01, 0.02, 0.02]
    print("[gpu] serve", len(reqs), "requests", flush=True)
    srv = serve.Server(capacity=3, budget_bytes=1 << 34, max_updates=4000, keep_results=True)
    res = srv.serve(reqs, arrivals)
    srv.close()
    assert res["summary"]["requests"] == 5 and res["summary"]["all_broke_through"]
    for rec, cfg in zip(res["records"], reqs):
        dev = torch.device("cuda:0")
        Kt = torch.from_numpy(inputs.permeability(cfg)).to(dev)
        st = torch.from_numpy(inputs.initial_saturation(cfg)).to(dev)
        r = binding.Run(cfg, Kt, st)
        r.start()
        n = r.advance(4000, True)
        assert n == rec["passes"]
        ux, uy = r.velocity()
        s = r.saturation()
        assert np.array_equal(to_np(ux), rec["state"][0]) and np.array_equal(to_np(uy), rec["state"][1])
        assert np.array_equal(to_np(s), rec["state"][2])
        assert r.stats()["te"] == rec["te"]
        r.close()


# Runs with equal decompositions step as one group: one launch per phase for all of them; the
# permeability, viscosities, cfl, eta and the epsilon norm may differ inside a group. Group A
# mixes MRCM and MPM-2P updates in the same step (small eta) and differs in those parameters,
# group B uses the text switch rule, group C the precision form, group D the first-order term;
# one run steps alone.
GROUPED = [
    # (seed, nx, ny, sub, ne, overrides, precision)
    (201, 32, 32, 8, 2, dict(sigma2=2.0, corr_len=0.2, mu_o=20.0, eta=0.01), 0),
    (202, 32, 32, 8, 2, dict(sigma2=2.0, corr_len=0.2, mu_o=35.0, eta=0.02, eps_norm="abs"), 0),
    (203, 32, 32, 8, 2, dict(sigma2=2.0, corr_len=0.2, mu_o=20.0, eta=0.01, cfl=0.4), 0),
    (204, 64, 48, 16, 4, dict(sigma2=3.0, corr_len=0.1, mu_o=50.0, eta=0.05, switch_rule="text"), 0),
    (205, 64, 48, 16, 4, dict(sigma2=3.0, corr_len=0.1, mu_o=50.0, eta=0.05, switch_rule="text"), 0),
    (206, 48, 32, 16, 4, dict(sigma2=2.0, corr_len=0.2, mu_o=30.0, eta=0.03), 1),
    (207, 48, 32, 16, 4, dict(sigma2=2.0, corr_len=0.2, mu_o=30.0, eta=0.03), 1),
    (208, 64, 64, 16, 8, dict(sigma2=4.0, corr_len=0.1, mu_o=100.0, eta=0.1), 0),
    (209, 32, 32, 8, 2, dict(sigma2=2.0, corr_len=0.2, mu_o=20.0, eta=0.01, mpm_order=1), 0),
    (210, 32, 32, 8, 2, dict(sigma2=2.0, corr_len=0.2, mu_o=25.0, eta=0.01, mpm_order=1), 0),
    (211, 32, 32, 8, 2, dict(sigma2=2.0, corr_len=0.2, mu_o=20.0, eta=0.01, iface_degree=1), 0),
    (212, 32, 32, 8, 2, dict(sigma2=2.0, corr_len=0.2, mu_o=30.0, eta=0.01, iface_degree=1), 0),
]


def _make_g(binding, p, stream=None, start=True):
    seed, nx, ny, sub, ne, kw, prec = p
    kw = dict(kw)
    sub_y, ne_y = kw.pop("sub_y", sub), kw.pop("ne_y", ne)
    cfg, K = inputs.random_problem(seed, nx, ny, sub, sub_y, ne, ne_y, **kw)
    dev = torch.device("cuda:0")
    Kt = torch.from_numpy(np.ascontiguousarray(K)).to(dev)
    st = torch.from_numpy(np.ascontiguousarray(inputs.initial_saturation(cfg))).to(dev)
    torch.cuda.synchronize()
    r = binding.Run(cfg, Kt, st, precision=prec, stream=stream)
    if start:
        r.start()
    return r


def _solo(binding, p, n):
    r = _make_g(binding, p)
    hist = []
    for _ in range(n):
        r.step()
        hist.append(r.stats()["last_branch"])
    out = _state(r)
    r.close()
    return out, hist


def test_grouped_batch_equals_solo(binding):
    nsteps = 12
    print("[gpu] grouped batch of", len(GROUPED), "runs,", nsteps, "steps", flush=True)
    solo = [_solo(binding, p, nsteps) for p in GROUPED]
    streams = [torch.cuda.Stream() for _ in GROUPED]
    runs = [_make_g(binding, p, s) for p, s in zip(GROUPED, streams)]
    b = binding.Batch(len(runs))
    for i, r in enumerate(runs):
        b.attach(i, r)
    for _ in range(nsteps):
        b.step()
    for r, (ref, _) in zip(runs, solo):
        _same(_state(r), ref)
    # group A took both branches within one step at least once
    hists = [h for _, h in solo[:3]]
    assert any(len({h[k] for h in hists}) == 2 for k in range(nsteps)), hists
    b.close()
    for r in runs:
        r.close()


def test_grouped_batch_parity_and_refill(binding):
    """Runs of one descriptor leave and rejoin the batch, so that their saturation buffers
    differ in parity (separate groups) and groups shrink and grow between steps; each run ends
    equal to its solo run with the same number of steps."""
    ps = GROUPED[:3]
    streams = [torch.cuda.Stream() for _ in ps]
    runs = [_make_g(binding, p, s) for p, s in zip(ps, streams)]
    n = [0, 0, 0]
    b = binding.Batch(3)
    for i, r in enumerate(runs):
        b.attach(i, r)
    for _ in range(3):
        b.step()
        n = [k + 1 for k in n]
    b.detach(0)
    b.step()                          # group of two
    n[1] += 1
    n[2] += 1
    b.attach(0, runs[0])              # back, one step behind: a group of its own parity
    for _ in range(2):
        b.step()
        n = [k + 1 for k in n]
    b.step([True, False, True])       # runs 0 and 2 (different parity)
    n[0] += 1
    n[2] += 1
    b.step([True, True, False])       # runs 0 and 1 (same parity again)
    n[0] += 1
    n[1] += 1
    got = [_state(r) for r in runs]
    b.close()
    for p, k, g in zip(ps, n, got):
        ref, _ = _solo(binding, p, k)
        _same(g, ref)
    for r in runs:
        r.close()


# eta = 0: many passes take the MRCM branch, in the same passes for every run of a group, which
# then share the update's launches
EVERY_PASS_MRCM = [
    (221, 32, 32, 8, 2, dict(sigma2=2.0, corr_len=0.2, mu_o=20.0, eta=0.0), 0),
    (222, 32, 32, 8, 2, dict(sigma2=2.5, corr_len=0.2, mu_o=30.0, eta=0.0), 0),
    (223, 32, 32, 8, 2, dict(sigma2=2.0, corr_len=0.15, mu_o=20.0, eta=0.0), 0),
    (224, 48, 32, 16, 4, dict(sigma2=2.0, corr_len=0.2, mu_o=30.0, eta=0.0), 1),
    (225, 48, 32, 16, 4, dict(sigma2=2.0, corr_len=0.2, mu_o=40.0, eta=0.0), 1),
    (226, 60, 30, 20, 4, dict(sigma2=2.0, corr_len=0.2, mu_o=30.0, eta=0.0, sub_y=10, ne_y=2), 0),
    (227, 60, 30, 20, 4, dict(sigma2=3.0, corr_len=0.2, mu_o=30.0, eta=0.0, sub_y=10, ne_y=2), 0),
]


def test_batch_start_and_grouped_mrcm_equal_solo(binding):
    """Runs attached before their start, started together (one launch per phase of the first
    MRCM update for each group of equal descriptors), then stepped: equal, bitwise, to the
    same runs started and stepped alone. Covers every phase of the MRCM update over a run table:
    the matrix-core basis and the many-line basis, the FP32 copies of the precision form, the
    factorisation and both first-order and linear-space groups, and passes in which every run of
    a group takes the MRCM branch."""
    ps = GROUPED + EVERY_PASS_MRCM
    nsteps = 4
    print("[gpu] batch start of", len(ps), "runs,", nsteps, "steps", flush=True)
    solo = [_solo(binding, p, nsteps) for p in ps]
    streams = [torch.cuda.Stream() for _ in ps]
    runs = [_make_g(binding, p, s, start=False) for p, s in zip(ps, streams)]
    b = binding.Batch(len(runs))
    for i, r in enumerate(runs):
        b.attach(i, r)
    b.start()
    for _ in range(nsteps):
        b.step()
    for p, r, (ref, hist) in zip(ps, runs, solo):
        got = _state(r)
        _same(got, ref)
        assert got[3]["error_word"] == 0
    # with the lagged rule and eta = 0 every other pass is an MRCM update, for all runs of a
    # group in the same passes
    hists = [hist for _, hist in solo[len(GROUPED):]]
    for hist in hists:
        assert sum(h == binding.FORCE_MRCM for h in hist) >= nsteps // 2, hist
    assert hists[0] == hists[1] == hists[2] and hists[3] == hists[4] and hists[5] == hists[6]
    b.close()
    for r in runs:
        r.close()


def test_batch_step_refuses_unstarted_runs(binding):
    p = GROUPED[0]
    r = _make_g(binding, p, torch.cuda.Stream(), start=False)
    b = binding.Batch(2)
    b.attach(0, r)
    with pytest.raises(binding.MpmError):
        b.step()
    b.start()
    b.step()
    assert r.stats()["te"] == 2
    b.close()
    r.close()


def _oracle_compare(cfg, orun, state, label):
    from .gpu_common import FP64_SAT_TOL, FP64_VEL_TOL, sat_rel_err, vel_face_err, vel_rel_err
    ux, uy, s, st = state
    ev = vel_rel_err(cfg, ux, uy, orun.ux, orun.uy)
    ef = vel_face_err(ux, uy, orun.ux, orun.uy)
    es = sat_rel_err(s, orun.s)
    print(f"    {label}: velocity {ev:.2e} (face {ef:.2e}), saturation {es:.2e}, T_e {st['te']} T_m {st['tm']}",
          flush=True)
    assert st["error_word"] == 0
    assert ev <= FP64_VEL_TOL and ef <= FP64_VEL_TOL and es <= FP64_SAT_TOL, (label, ev, ef, es)
    assert st["te"] == orun.n and st["tm"] == orun.ell + 1, label
    assert abs(st["pvi"] - orun.pvi) <= 1e-10 * orun.pvi


def test_batch_classes_match_oracle(binding):
    """One realisation of each class of the batched workload (64^2 in 8^2 subdomains, 128^2 in
    16^2, 256^2 in 32^2, 4 elements per side, log-variance 4, M = 100) stepped together in one batch
    for 30 passes of Algorithm 1 against the FP64 oracle run alone on the same inputs (the 64^2
    run with eta = 0.02, so that its switch takes basis updates inside the window)."""
    from oracle import splitting
    nsteps = 30
    cfgs = inputs.batch_workload(3)
    cfgs[0]["eta"] = 0.02
    dev = torch.device("cuda:0")
    streams = [torch.cuda.Stream() for _ in cfgs]
    runs = []
    for c, stream in zip(cfgs, streams):
        Kt = torch.from_numpy(inputs.permeability(c)).to(dev)
        st = torch.from_numpy(inputs.initial_saturation(c)).to(dev)
        torch.cuda.synchronize()
        runs.append(binding.Run(c, Kt, st, stream=stream))
    b = binding.Batch(len(runs))
    for i, r in enumerate(runs):
        b.attach(i, r)
    b.start()
    for _ in range(nsteps):
        b.step()
    b.close()
    states = [_state(r) for r in runs]
    for r in runs:
        r.close()
    for c, state in zip(cfgs, states):
        print(f"[gpu] batch class {c['nx']}^2 (subdomains {c['sub_x']}^2) against the oracle", flush=True)
        orun = splitting.simulate(c, inputs.permeability(c), inputs.initial_saturation(c), nsteps + 1)
        _oracle_compare(c, orun, state, f"{c['nx']}^2")
    assert states[0][3]["tm"] > 1, "no basis update in the window"


@pytest.mark.timeout(600)
def test_served_512_request_matches_oracle(binding):
    """A 512^2 request of the serving workload (32 x 32 subdomains of 16^2, 4 elements per side)
    served beside a 128^2 and a 256^2 request through the continuous-batching server, stopped
    after 8 passes, against the FP64 oracle run alone on the same inputs."""
    from oracle import splitting
    from paper_2103_11050_amd import serve
    reqs = inputs.serve_requests(24, (128, 256, 512))
    pick = {}
    for c in reqs:
        pick.setdefault(c["nx"], c)
    sel = [pick[128], pick[256], pick[512]]
    npass = 8
    srv = serve.Server(3, 8 << 30, max_updates=npass, keep_results=True)
    res = srv.serve(sel, [0.0, 0.0, 0.0])
    srv.close()
    rec = res["records"][2]
    assert rec["nx"] == 512 and rec["passes"] == npass
    c = sel[2]
    print(f"[gpu] served 512^2 request (M = {c['mu_o']:.1f}, log-variance {c['sigma2']:.2f}) against the oracle",
          flush=True)
    orun = splitting.simulate(c, inputs.permeability(c), inputs.initial_saturation(c), npass + 1)
    ux, uy, s = rec["state"]
    st = {"te": rec["te"], "tm": rec["tm"], "pvi": rec["pvi"], "error_word": rec["error_word"]}
    _oracle_compare(c, orun, (ux, uy, s, st), "512^2 served")
