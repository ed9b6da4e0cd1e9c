"""Thin ctypes binding of the C ABI declared in include/mpm2p.h.

Argument marshalling only: every step of the method runs in the HIP library. PyTorch
provides device memory (the workspace and the field tensors) and the stream. Loading fails
loudly when the compiled library is missing.
"""
from __future__ import annotations

import ctypes
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmpm2p.so")

MPM_OK, MPM_EINVAL, MPM_ENOMEM, MPM_ENOTSPD, MPM_ESINGULAR, MPM_ENONFINITE, MPM_EHIP, MPM_ESTATE = 0, -1, -2, -3, -4, -5, -6, -7
MPM_ENOCONV = -8
EPS_REL, EPS_ABS = 0, 1
SWITCH_ALG1, SWITCH_TEXT = 0, 1
PREC_FP64, PREC_FP32_REFINE = 0, 1
AUTO, FORCE_MPM, FORCE_MRCM = -1, 0, 1
ABI_VERSION = 3
# refinement target of the precision form when the configuration names none
REFINE_RTOL_DEFAULT = 1e-10


class Desc(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_int32),
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("lx", ctypes.c_double), ("ly", ctypes.c_double),
        ("sub_x", ctypes.c_int32), ("sub_y", ctypes.c_int32),
        ("ne_x", ctypes.c_int32), ("ne_y", ctypes.c_int32),
        ("alpha", ctypes.c_double), ("eta", ctypes.c_double),
        ("eps_norm", ctypes.c_int32), ("switch_rule", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("cn", ctypes.c_int32),
        ("mu_w", ctypes.c_double), ("mu_o", ctypes.c_double),
        ("bc_kind", ctypes.c_int32 * 4), ("bc_value", ctypes.c_double * 4),
        ("s_inj", ctypes.c_double), ("cfl", ctypes.c_double),
        ("breakthrough_cut", ctypes.c_double),
        ("mpm_order", ctypes.c_int32), ("iface_degree", ctypes.c_int32),
        ("refine_rtol", ctypes.c_double),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("te", ctypes.c_int64), ("tm", ctypes.c_int64), ("n_transport", ctypes.c_int64),
        ("eps", ctypes.c_double), ("t", ctypes.c_double), ("pvi", ctypes.c_double),
        ("water_cut", ctypes.c_double), ("dt", ctypes.c_double),
        ("breakthrough", ctypes.c_int32), ("last_branch", ctypes.c_int32),
        ("error_word", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


# every symbol the header declares, with its signature
_SIGS = {
    "mpm_workspace_size": (ctypes.c_int32, [ctypes.POINTER(Desc), ctypes.POINTER(ctypes.c_size_t)]),
    "mpm_create": (ctypes.c_int32, [ctypes.POINTER(Desc), ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                    ctypes.POINTER(ctypes.c_void_p)]),
    "mpm_create_static": (ctypes.c_int32, [ctypes.POINTER(Desc), ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "mpm_set_fields": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "mpm_start": (ctypes.c_int32, [ctypes.c_void_p]),
    "mpm_transport": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32]),
    "mpm_velocity_update": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32]),
    "mpm_step": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32]),
    "mpm_get_velocity": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "mpm_get_saturation": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p]),
    "mpm_get_stats": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(Stats)]),
    "mpm_destroy": (ctypes.c_int32, [ctypes.c_void_p]),
    "mpm_status_str": (ctypes.c_char_p, [ctypes.c_int32]),
    "mpm_plan_info": (ctypes.c_int32, [ctypes.c_void_p] + [ctypes.POINTER(ctypes.c_int64)] * 4),
    "mpm_plan_solve_bytes": (ctypes.c_int32, [ctypes.c_void_p] + [ctypes.POINTER(ctypes.c_int64)] * 3),
    "mpm_plan_fused_bytes": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]
                             + [ctypes.POINTER(ctypes.c_int64)] * 2),
    "mpm_advance": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "mpm_last_error": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_char_p, ctypes.c_size_t]),
    "mpm_batch_create": (ctypes.c_int32, [ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p)]),
    "mpm_batch_attach": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "mpm_batch_detach": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32]),
    "mpm_batch_step": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "mpm_batch_start": (ctypes.c_int32, [ctypes.c_void_p]),
    "mpm_batch_destroy": (ctypes.c_int32, [ctypes.c_void_p]),
    "mpm_tune": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                  ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_double)]),
    "mpm_profile": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32)]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Loads the HIP library; raises RuntimeError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library {path} is missing: build it with `python -m paper_2103_11050_amd.build`")
    # PyTorch brings its own HIP runtime; load it first so that the library binds to the same
    # runtime instance as the tensors and streams it is given (one runtime per process)
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class MpmError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = load().mpm_status_str(status).decode()
        super().__init__(f"{where}: {msg} ({status})")


def _check(status: int, where: str):
    if status != MPM_OK:
        raise MpmError(status, where)


_EPS = {"rel": EPS_REL, "abs": EPS_ABS}
_SWITCH = {"alg1": SWITCH_ALG1, "text": SWITCH_TEXT}


def make_desc(cfg: dict, precision: int = PREC_FP64) -> Desc:
    d = Desc()
    d.abi_version = ABI_VERSION
    d.nx, d.ny = cfg["nx"], cfg["ny"]
    d.lx, d.ly = cfg["lx"], cfg["ly"]
    d.sub_x, d.sub_y = cfg["sub_x"], cfg["sub_y"]
    d.ne_x, d.ne_y = cfg["ne_x"], cfg["ne_y"]
    d.alpha = cfg["alpha"]
    d.eta = float(cfg["eta"])
    d.eps_norm = _EPS[cfg.get("eps_norm", "rel")]
    d.switch_rule = _SWITCH[cfg.get("switch_rule", "alg1")]
    d.precision = precision
    d.cn = cfg["cn"]
    d.mu_w, d.mu_o = cfg["mu_w"], cfg["mu_o"]
    for k in range(4):
        d.bc_kind[k] = int(cfg["bc_kind"][k])
        d.bc_value[k] = float(cfg["bc_value"][k])
    d.s_inj = cfg["s_inj"]
    d.cfl = cfg["cfl"]
    d.breakthrough_cut = cfg["breakthrough_cut"]
    d.mpm_order = int(cfg.get("mpm_order", 0))
    d.iface_degree = int(cfg.get("iface_degree", 0))
    d.refine_rtol = float(cfg.get("refine_rtol", REFINE_RTOL_DEFAULT))
    return d


def workspace_size(cfg: dict, precision: int = PREC_FP64) -> int:
    d = make_desc(cfg, precision)
    n = ctypes.c_size_t()
    _check(load().mpm_workspace_size(ctypes.byref(d), ctypes.byref(n)), "mpm_workspace_size")
    return n.value


def _ptr(t) -> int:
    return 0 if t is None else t.data_ptr()


class Run:
    """One MPM-2P run on the current device (thin wrapper of mpm_run)."""

    def __init__(self, cfg: dict, K, s0, q=None, precision: int = PREC_FP64, stream=None, static=False):
        """static: the workspace is the library's own device array (mpm_create_static) instead
        of a tensor allocated here."""
        import torch
        lib = load()
        self.cfg = cfg
        self.device = K.device
        self.desc = make_desc(cfg, precision)
        n = ctypes.c_size_t()
        _check(lib.mpm_workspace_size(ctypes.byref(self.desc), ctypes.byref(n)), "mpm_workspace_size")
        self.ws_bytes = n.value
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        if static:
            self.ws = None
            st = lib.mpm_create_static(ctypes.byref(self.desc), ctypes.c_void_p(self.stream.cuda_stream),
                                       ctypes.byref(h))
        else:
            self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
            aligned = (self.ws.data_ptr() + 255) & ~255
            st = lib.mpm_create(ctypes.byref(self.desc), ctypes.c_void_p(aligned), ctypes.c_size_t(self.ws_bytes),
                                ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if st != MPM_OK:
            buf = ctypes.create_string_buffer(512)
            lib.mpm_last_error(None, buf, 512)
            _check(st, ("mpm_create_static" if static else "mpm_create") + " (" + buf.value.decode() + ")")
        self.h = h
        self._keep = (K, s0, q)
        # the inputs were written on the caller's current stream
        cur = torch.cuda.current_stream(self.device)
        if self.stream != cur:
            self.stream.wait_stream(cur)
        _check(lib.mpm_set_fields(self.h, ctypes.c_void_p(_ptr(K)), ctypes.c_void_p(_ptr(q)),
                                  ctypes.c_void_p(_ptr(s0))), "mpm_set_fields")

    def start(self):
        _check(load().mpm_start(self.h), "mpm_start")

    def step(self, force: int = AUTO):
        _check(load().mpm_step(self.h, force), "mpm_step")

    def advance(self, max_updates: int, stop_at_breakthrough: bool = True) -> int:
        done = ctypes.c_int32()
        _check(load().mpm_advance(self.h, max_updates, int(stop_at_breakthrough), ctypes.byref(done)), "mpm_advance")
        return done.value

    def last_error(self) -> str:
        buf = ctypes.create_string_buffer(512)
        _check(load().mpm_last_error(self.h, buf, 512), "mpm_last_error")
        return buf.value.decode()

    def transport(self, nsteps: int):
        _check(load().mpm_transport(self.h, nsteps), "mpm_transport")

    def velocity_update(self, force: int = AUTO):
        _check(load().mpm_velocity_update(self.h, force), "mpm_velocity_update")

    def velocity(self):
        import torch
        nx, ny = self.cfg["nx"], self.cfg["ny"]
        ux = torch.empty((ny, nx + 1), dtype=torch.float64, device=self.device)
        uy = torch.empty((ny + 1, nx), dtype=torch.float64, device=self.device)
        _check(load().mpm_get_velocity(self.h, ctypes.c_void_p(ux.data_ptr()), ctypes.c_void_p(uy.data_ptr())),
               "mpm_get_velocity")
        self._hand_over(ux, uy)
        return ux, uy

    def _hand_over(self, *ts):
        """Outputs written on the run's stream become usable on the caller's current stream."""
        import torch
        cur = torch.cuda.current_stream(self.device)
        if self.stream != cur:
            for t in ts:
                t.record_stream(self.stream)
            cur.wait_stream(self.stream)

    def saturation(self):
        import torch
        s = torch.empty((self.cfg["ny"], self.cfg["nx"]), dtype=torch.float64, device=self.device)
        _check(load().mpm_get_saturation(self.h, ctypes.c_void_p(s.data_ptr())), "mpm_get_saturation")
        self._hand_over(s)
        return s

    def stats(self) -> dict:
        st = Stats()
        _check(load().mpm_get_stats(self.h, ctypes.byref(st)), "mpm_get_stats")
        return {k: getattr(st, k) for k, _ in Stats._fields_ if k != "reserved"}

    def plan_info(self) -> dict:
        v = [ctypes.c_int64() for _ in range(4)]
        _check(load().mpm_plan_info(self.h, *[ctypes.byref(x) for x in v]), "mpm_plan_info")
        return dict(n_sub=v[0].value, n_iface=v[1].value, n_nodes=v[2].value, n_levels=v[3].value)

    def solve_bytes(self) -> dict:
        v = [ctypes.c_int64() for _ in range(3)]
        _check(load().mpm_plan_solve_bytes(self.h, *[ctypes.byref(x) for x in v]), "mpm_plan_solve_bytes")
        return dict(fwd=v[0].value, bwd=v[1].value, front=v[2].value)

    def fused_bytes(self) -> dict:
        """Bytes of the bottom tree levels swept by one launch per direction (mpm_plan_fused_bytes)."""
        lv = ctypes.c_int32()
        v = [ctypes.c_int64() for _ in range(2)]
        _check(load().mpm_plan_fused_bytes(self.h, ctypes.byref(lv), *[ctypes.byref(x) for x in v]),
               "mpm_plan_fused_bytes")
        return dict(levels=lv.value, fwd=v[0].value, bwd=v[1].value)

    def tune(self, reps: int = 5) -> dict:
        """Autotunes the interface-sweep launch shapes of this run (mpm_tune)."""
        cap = 3 * 128
        shapes = (ctypes.c_int32 * cap)()
        n = ctypes.c_int32()
        t0, t1 = ctypes.c_double(), ctypes.c_double()
        _check(load().mpm_tune(self.h, reps, cap, shapes, ctypes.byref(n), ctypes.byref(t0), ctypes.byref(t1)),
               "mpm_tune")
        k = min(n.value, cap // 3)
        return {"ms_rule": t0.value, "ms_tuned": t1.value,
                "shapes": [tuple(shapes[3 * i:3 * i + 3]) for i in range(k)]}

    def profile(self, enable: int = 1, reset: bool = True) -> dict:
        """Kernel-class timings (mpm_profile): enable 1 times the phases, 2 also the fused sweep
        launches, 0 stops; returns what was collected since the last reset."""
        cap = 64
        names = (ctypes.c_char_p * cap)()
        ms = (ctypes.c_double * cap)()
        cnt = (ctypes.c_int64 * cap)()
        n = ctypes.c_int32()
        _check(load().mpm_profile(self.h, int(enable), int(reset), cap, names, ms, cnt, ctypes.byref(n)),
               "mpm_profile")
        return {names[i].decode(): (ms[i], cnt[i]) for i in range(n.value)}

    def close(self):
        if getattr(self, "h", None):
            st = load().mpm_destroy(self.h)
            self.h = None
            _check(st, "mpm_destroy")

    def __del__(self):
        try:
            if getattr(self, "h", None):
                load().mpm_destroy(self.h)
                self.h = None
        except Exception:
            pass


def header_symbols(header_path: str) -> list[str]:
    """Function names declared in the public header (used by the ABI test)."""
    import re
    txt = open(header_path).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:mpm_status|const char\s*\*)\s*(mpm_[a-z_]+)\s*\(", txt, flags=re.M)))


class Batch:
    """Slots of runs stepped together (thin wrapper of mpm_batch); runs attached before their
    start are started by `start()`. Give each run its own stream so that their work overlaps on
    the device."""

    def __init__(self, capacity: int):
        h = ctypes.c_void_p()
        _check(load().mpm_batch_create(capacity, ctypes.byref(h)), "mpm_batch_create")
        self.h = h
        self.capacity = capacity
        self.runs = [None] * capacity

    def attach(self, slot: int, run: "Run"):
        _check(load().mpm_batch_attach(self.h, slot, run.h), "mpm_batch_attach")
        self.runs[slot] = run

    def detach(self, slot: int):
        _check(load().mpm_batch_detach(self.h, slot), "mpm_batch_detach")
        self.runs[slot] = None

    def start(self):
        """Starts the attached runs that are not started, those with equal descriptors together."""
        _check(load().mpm_batch_start(self.h), "mpm_batch_start")

    def step(self, active=None):
        """One pass for every filled (and active) slot; returns the per-slot breakthrough flags."""
        bt = (ctypes.c_uint8 * self.capacity)()
        act = None
        if active is not None:
            act = (ctypes.c_uint8 * self.capacity)(*[1 if a else 0 for a in active])
        _check(load().mpm_batch_step(self.h, act, bt), "mpm_batch_step")
        return [bool(x) for x in bt]

    def close(self):
        if self.h:
            load().mpm_batch_destroy(self.h)
            self.h = None
