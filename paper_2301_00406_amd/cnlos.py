"""Python binding of libcnlos (ctypes).  Argument marshalling only: every step
of the reconstruction runs in the HIP library; PyTorch provides device memory
and the stream.  The library must be built (``build_lib.build()``); there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_double, c_int32, c_uint8, c_uint64, c_void_p

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libcnlos.so")

OK, EINVAL, EUNSUPPORTED, ENOMEM, EHIP, ESTATE, EBACKTRACK, ENONFINITE = range(8)
MODEL_OPERATOR, MODEL_OBJECT, MODEL_DUAL = 0, 1, 2
PHI_TSC, PHI_TAC, PHI_TRV = 0, 1, 2
FALLOFF_COMPENSATED, FALLOFF_LITERAL = 0, 1
(FIELD_U, FIELD_UBAR, FIELD_V, FIELD_LAM, FIELD_PHI, FIELD_AU, FIELD_AU_PREV, FIELD_TAU0,
 FIELD_TAU, FIELD_TAUBAR, FIELD_W, FIELD_LAM2, FIELD_F, FIELD_LAM3, FIELD_PHI_TAU) = range(15)
VECTOR_FIELDS = {FIELD_V, FIELD_LAM, FIELD_W, FIELD_LAM2}
KERNEL_KINDS = ["t_fwd_conv", "plane_conv", "t_inv_conv", "t_fwd_solve", "plane_solve",
                "t_inv_solve", "field", "post", "control", "other"]

_STATUS_NAMES = {OK: "CNLOS_OK", EINVAL: "CNLOS_EINVAL", EUNSUPPORTED: "CNLOS_EUNSUPPORTED",
                 ENOMEM: "CNLOS_ENOMEM", EHIP: "CNLOS_EHIP", ESTATE: "CNLOS_ESTATE",
                 EBACKTRACK: "CNLOS_EBACKTRACK", ENONFINITE: "CNLOS_ENONFINITE"}


class Config(ctypes.Structure):
    _fields_ = [
        ("nx", c_int32), ("ny", c_int32), ("nt", c_int32), ("model", c_int32),
        ("wall_w_m", c_double), ("wall_h_m", c_double), ("bin_ps", c_double),
        ("phi", c_int32), ("falloff", c_int32),
        ("a_u", c_double), ("b_u", c_double), ("a_tau", c_double), ("b_tau", c_double),
        ("warm_a", c_double), ("warm_b", c_double), ("mu", c_double),
        ("mu1", c_double), ("mu2", c_double), ("mu3", c_double), ("lambda_", c_double),
        ("eta_curv", c_double),
        ("max_iters", c_int32), ("init_iters", c_int32),
        ("eps_stop", c_double),
        ("backtracking", c_int32), ("bt_max_trials", c_int32),
        ("L0", c_double), ("L0_dual", c_double), ("bt_factor", c_double),
        ("power_iters", c_int32), ("fista_restart", c_int32),
    ]


class Report(ctypes.Structure):
    _fields_ = [("iters_done", c_int32), ("total_iters", c_int32), ("stopped_early", c_int32),
                ("bt_rejects", c_int32), ("L_final", c_double), ("energy", c_double),
                ("primal_res", c_double), ("dual_res", c_double), ("status", c_int32),
                ("reserved", c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("L0_obj", c_double), ("L0_dual", c_double), ("L", c_double), ("t", c_double),
                ("beta", c_double), ("meas_scale", c_double), ("energy_prev", c_double),
                ("iter", c_int32), ("stage", c_int32), ("bt_rejects", c_int32),
                ("has_measurement", c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("cfg", Config), ("mask_host", POINTER(c_uint8)), ("tau0_dev", c_void_p),
                ("out_dev", c_void_p), ("id", ctypes.c_int64)]


class Completion(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("status", c_int32), ("iters", c_int32),
                ("energy", c_double), ("queued_steps", c_double), ("served_steps", c_double)]


class Plan(ctypes.Structure):
    _fields_ = [("conv_row_pad", c_int32), ("solve_row_pad", c_int32), ("tuned", c_int32),
                ("reserved", c_int32), ("conv_plane_us", c_double * 3),
                ("solve_plane_us", c_double * 3)]


def _plan_dict(pl):
    return {"conv_row_pad": pl.conv_row_pad, "solve_row_pad": pl.solve_row_pad,
            "tuned": bool(pl.tuned), "conv_plane_us": list(pl.conv_plane_us),
            "solve_plane_us": list(pl.solve_plane_us)}


class NcGeometry(ctypes.Structure):
    _fields_ = [("n", c_int32), ("m", c_int32), ("wall_m", c_double), ("bin_ps", c_double),
                ("illum_x_m", c_double), ("illum_y_m", c_double), ("literal", c_int32)]


class CnlosError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None


def load() -> ctypes.CDLL:
    """Load libcnlos.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "paper_2301_00406_amd.build_lib.build()")
    lib = ctypes.CDLL(LIB_PATH)
    P = c_void_p
    sig = {
        "cnlos_version": ([], ctypes.c_char_p),
        "cnlos_last_error": ([], ctypes.c_char_p),
        "cnlos_config_default": ([POINTER(Config)], None),
        "cnlos_validate": ([POINTER(Config), POINTER(c_uint8)], c_int32),
        "cnlos_workspace_bytes": ([POINTER(Config), POINTER(c_uint64)], c_int32),
        "cnlos_create": ([POINTER(Config), POINTER(c_uint8), P, c_uint64, P, POINTER(P)], c_int32),
        "cnlos_set_measurement": ([P, P], c_int32),
        "cnlos_apply_A": ([P, P, P, c_int32], c_int32),
        "cnlos_apply_AT": ([P, P, P, c_int32], c_int32),
        "cnlos_apply_A_noalloc": ([POINTER(Config), POINTER(c_uint8), P, P, c_int32, P], c_int32),
        "cnlos_run": ([P, c_int32, POINTER(Report)], c_int32),
        "cnlos_reset": ([P], c_int32),
        "cnlos_get_volume": ([P, P], c_int32),
        "cnlos_get_signal": ([P, P], c_int32),
        "cnlos_get_field": ([P, c_int32, P], c_int32),
        "cnlos_set_field": ([P, c_int32, P], c_int32),
        "cnlos_get_info": ([P, POINTER(Info)], c_int32),
        "cnlos_set_info": ([P, POINTER(Info)], c_int32),
        "cnlos_get_log": ([P, POINTER(c_double), c_int32, POINTER(c_int32)], c_int32),
        "cnlos_profile_enable": ([P, ctypes.c_uint32], c_int32),
        "cnlos_profile_read": ([P, POINTER(c_double), POINTER(ctypes.c_int64), c_int32], c_int32),
        "cnlos_destroy": ([P], c_int32),
        "cnlos_batch_workspace_bytes": ([POINTER(Config), c_int32, POINTER(c_uint64)], c_int32),
        "cnlos_batch_create": ([POINTER(Config), c_int32, POINTER(POINTER(c_uint8)), P, c_uint64, P,
                                POINTER(P)], c_int32),
        "cnlos_batch_member": ([P, c_int32, POINTER(P)], c_int32),
        "cnlos_batch_run": ([P, c_int32, POINTER(Report)], c_int32),
        "cnlos_batch_run_many": ([POINTER(P), c_int32, c_int32, POINTER(POINTER(Report))], c_int32),
        "cnlos_batch_destroy": ([P], c_int32),
        "cnlos_server_create": ([P, c_uint64, c_int32, c_int32, POINTER(P)], c_int32),
        "cnlos_server_submit": ([P, POINTER(Request)], c_int32),
        "cnlos_server_step": ([P, POINTER(c_int32), POINTER(c_int32)], c_int32),
        "cnlos_server_poll": ([P, POINTER(Completion), c_int32, POINTER(c_int32)], c_int32),
        "cnlos_server_fail_next_groups": ([P, c_int32], c_int32),
        "cnlos_server_usage": ([P, POINTER(c_uint64), POINTER(c_int32)], c_int32),
        "cnlos_server_destroy": ([P], c_int32),
        "cnlos_tune": ([P, POINTER(Plan)], c_int32),
        "cnlos_get_plan": ([P, POINTER(Plan)], c_int32),
        "cnlos_set_plan": ([P, POINTER(Plan)], c_int32),
        "cnlos_nc_validate": ([POINTER(NcGeometry)], c_int32),
        "cnlos_nc_apply": ([POINTER(NcGeometry), P, P, P], c_int32),
        "cnlos_nc_apply_T": ([POINTER(NcGeometry), P, P, P], c_int32),
        "cnlos_nc_midpoint": ([POINTER(NcGeometry), POINTER(c_double), POINTER(c_double),
                               POINTER(c_double)], c_int32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def last_error() -> str:
    return load().cnlos_last_error().decode()


def check(status: int) -> None:
    if status != OK:
        raise CnlosError(status, last_error())


def default_config(**overrides) -> Config:
    cfg = Config()
    load().cnlos_config_default(byref(cfg))
    for k, v in overrides.items():
        key = "lambda_" if k == "lam" else k
        if not hasattr(cfg, key):
            raise AttributeError(k)
        setattr(cfg, key, v)
    return cfg


def validate(cfg: Config, mask=None) -> int:
    lib = load()
    if mask is None:
        return lib.cnlos_validate(byref(cfg), None)
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    return lib.cnlos_validate(byref(cfg), m.ctypes.data_as(POINTER(c_uint8)))


def workspace_bytes(cfg: Config) -> int:
    n = c_uint64()
    check(load().cnlos_workspace_bytes(byref(cfg), byref(n)))
    return int(n.value)


def apply_A_noalloc(cfg: Config, mask, u, out, masked=False, stream=None):
    """tau = A u (or D A u) for a configuration, with no handle and no
    workspace: the library's static scratch holds the operator (the entry
    point for callers that cannot allocate).  u and out are contiguous float32
    [nx][ny][nt] tensors on the current device."""
    import torch
    lib = load()
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    shape = (cfg.nx, cfg.ny, cfg.nt)
    dev = torch.device("cuda", torch.cuda.current_device())
    _dev_f32(u, shape, dev)
    _dev_f32(out, shape, dev)
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    check(lib.cnlos_apply_A_noalloc(byref(cfg), m.ctypes.data_as(POINTER(c_uint8)),
                                    c_void_p(u.data_ptr()), c_void_p(out.data_ptr()),
                                    int(bool(masked)), c_void_p(st.cuda_stream)))
    return out


def nc_geometry(n, m, wall_m, bin_ps, illum, literal=True) -> NcGeometry:
    """Geometry of the non-confocal operator: n x n detectors, m bins, a square
    wall of extent wall_m, bin width bin_ps, illuminated wall point illum."""
    return NcGeometry(int(n), int(m), float(wall_m), float(bin_ps), float(illum[0]),
                      float(illum[1]), int(bool(literal)))


def nc_validate(g: NcGeometry) -> int:
    return load().cnlos_nc_validate(byref(g))


def _nc_call(fn, g, src, out, stream):
    import torch
    shape = (g.n, g.n, g.m)
    dev = src.device if isinstance(src, torch.Tensor) else None
    if dev is None or dev.type != "cuda":
        raise ValueError("expected CUDA tensors")
    a = _dev_f32(src, shape, dev)
    b = _dev_f32(out, shape, dev)
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    with torch.cuda.device(dev):
        check(fn(byref(g), a, b, c_void_p(st.cuda_stream)))
    return out


def nc_apply(g: NcGeometry, u, out=None, stream=None):
    """tau = A_nc u (non-confocal model by direct summation); u and out are
    contiguous float32 [n][n][m] device tensors.  Asynchronous on the stream."""
    import torch
    out = torch.empty_like(u) if out is None else out
    return _nc_call(load().cnlos_nc_apply, g, u, out, stream)


def nc_apply_T(g: NcGeometry, tau, out=None, stream=None):
    """u = A_nc^T tau (the transpose)."""
    import torch
    out = torch.empty_like(tau) if out is None else out
    return _nc_call(load().cnlos_nc_apply_T, g, tau, out, stream)


def nc_midpoint(g: NcGeometry):
    """Midpoint approximation: (wall extent of the confocal grid, (x, y) of its
    centre) for reconstructing the transients with the confocal solver."""
    w, cx, cy = c_double(), c_double(), c_double()
    check(load().cnlos_nc_midpoint(byref(g), byref(w), byref(cx), byref(cy)))
    return w.value, (cx.value, cy.value)


def _dev_f32(t, shape, device):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if t.dtype != torch.float32 or t.device != device or not t.is_contiguous():
        raise ValueError(f"expected a contiguous float32 tensor on {device}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"expected shape {tuple(shape)}, got {tuple(t.shape)}")
    return c_void_p(t.data_ptr())


class Problem:
    """One reconstruction problem in a device workspace owned by this object."""

    def __init__(self, cfg: Config, mask, device=None, stream=None, workspace=None, _member=None):
        import torch
        self._lib = load()
        self._owned = _member is None
        if _member is not None:           # a batch member: the batch owns handle and memory
            h, owner = _member
            self.cfg = cfg
            self.device = owner.device
            self.shape = (cfg.nx, cfg.ny, cfg.nt)
            self.workspace = owner.workspace
            self.stream = owner.stream
            self.mask = np.ascontiguousarray(mask, dtype=np.uint8)
            self._owner = owner
            self._h = h
            return
        self.cfg = cfg
        self.device = torch.device(device if device is not None else "cuda")
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.shape = (cfg.nx, cfg.ny, cfg.nt)
        nbytes = workspace_bytes(cfg)
        if workspace is None:
            workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        elif workspace.numel() < nbytes:
            raise ValueError("workspace too small")
        self.workspace = workspace
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        m = np.ascontiguousarray(mask, dtype=np.uint8)
        if m.shape != (cfg.nx, cfg.ny):
            raise ValueError(f"mask must be {(cfg.nx, cfg.ny)}")
        self.mask = m
        h = c_void_p()
        with torch.cuda.device(self.device):
            st = self._lib.cnlos_create(byref(cfg), m.ctypes.data_as(POINTER(c_uint8)),
                                        c_void_p(workspace.data_ptr()), c_uint64(nbytes),
                                        c_void_p(self.stream.cuda_stream), byref(h))
        self._h = h
        if st != OK:
            msg = last_error()
            self.close()
            raise CnlosError(st, msg)

    # -- lifetime
    def close(self):
        if (getattr(self, "_owned", False) and getattr(self, "_h", None) is not None
                and self._h.value is not None):
            self._lib.cnlos_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _vol(self, t):
        return _dev_f32(t, self.shape, self.device)

    def _empty(self, shape=None):
        import torch
        return torch.empty(shape or self.shape, dtype=torch.float32, device=self.device)

    # -- operator
    def set_measurement(self, tau0):
        check(self._lib.cnlos_set_measurement(self._h, self._vol(tau0)))

    def apply_A(self, u, masked=False, out=None):
        out = self._empty() if out is None else out
        check(self._lib.cnlos_apply_A(self._h, self._vol(u), self._vol(out), int(bool(masked))))
        return out

    def apply_AT(self, tau, masked=False, out=None):
        out = self._empty() if out is None else out
        check(self._lib.cnlos_apply_AT(self._h, self._vol(tau), self._vol(out), int(bool(masked))))
        return out

    # -- solver
    def run(self, iters=0):
        rep = Report()
        st = self._lib.cnlos_run(self._h, int(iters), byref(rep))
        if st != OK:
            raise CnlosError(st, last_error())
        return {f: getattr(rep, f) for f, _ in Report._fields_}

    def run_status(self, iters=0):
        """Like run() but returns (status, report) instead of raising."""
        rep = Report()
        st = self._lib.cnlos_run(self._h, int(iters), byref(rep))
        return st, {f: getattr(rep, f) for f, _ in Report._fields_}

    def reset(self):
        check(self._lib.cnlos_reset(self._h))

    def volume(self):
        out = self._empty()
        check(self._lib.cnlos_get_volume(self._h, self._vol(out)))
        return out

    def signal(self):
        out = self._empty()
        check(self._lib.cnlos_get_signal(self._h, self._vol(out)))
        return out

    def _field_shape(self, field):
        return ((3,) + self.shape) if field in VECTOR_FIELDS else self.shape

    def get_field(self, field):
        shp = self._field_shape(field)
        out = self._empty(shp)
        check(self._lib.cnlos_get_field(self._h, int(field), _dev_f32(out, shp, self.device)))
        return out

    def set_field(self, field, src):
        shp = self._field_shape(field)
        check(self._lib.cnlos_set_field(self._h, int(field), _dev_f32(src, shp, self.device)))

    def info(self):
        inf = Info()
        check(self._lib.cnlos_get_info(self._h, byref(inf)))
        return {f: getattr(inf, f) for f, _ in Info._fields_}

    def set_info(self, d):
        inf = Info()
        for f, _ in Info._fields_:
            if f in d:
                setattr(inf, f, d[f])
        check(self._lib.cnlos_set_info(self._h, byref(inf)))

    def tune(self):
        """Measure the plane kernels' candidate layouts on this problem, keep the
        fastest (also for later problems of this shape) and return the plan
        with the measured times.  Resets the iteration state."""
        pl = Plan()
        check(self._lib.cnlos_tune(self._h, byref(pl)))
        return _plan_dict(pl)

    def plan(self):
        pl = Plan()
        check(self._lib.cnlos_get_plan(self._h, byref(pl)))
        return _plan_dict(pl)

    def set_plan(self, conv_row_pad, solve_row_pad):
        pl = Plan()
        pl.conv_row_pad, pl.solve_row_pad = int(conv_row_pad), int(solve_row_pad)
        check(self._lib.cnlos_set_plan(self._h, byref(pl)))

    def profile_enable(self, kinds):
        """Time every later launch of the named kernel kinds with HIP events."""
        mask = 0
        for k in kinds:
            mask |= 1 << KERNEL_KINDS.index(k)
        check(self._lib.cnlos_profile_enable(self._h, mask))

    def profile_read(self, reset=True):
        n = len(KERNEL_KINDS)
        ms = (c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        check(self._lib.cnlos_profile_read(self._h, ms, cnt, int(bool(reset))))
        return {k: (ms[i], int(cnt[i])) for i, k in enumerate(KERNEL_KINDS) if cnt[i]}

    def log(self, cap=4096):
        buf = np.zeros((cap, 6), dtype=np.float64)
        n = c_int32()
        check(self._lib.cnlos_get_log(self._h, buf.ctypes.data_as(POINTER(c_double)), cap, byref(n)))
        return buf[: n.value].copy()


def _report_dict(rep):
    return {f: getattr(rep, f) for f, _ in Report._fields_}


class Batch:
    """Problems of one shape and one set of solver parameters that advance
    together: every kernel of an iteration is one launch for all members."""

    def __init__(self, cfgs, masks, device=None, stream=None):
        import torch
        self._lib = load()
        self._h = None
        cfgs = list(cfgs)
        if len(cfgs) != len(masks) or not cfgs:
            raise ValueError("need one mask per config")
        self.device = torch.device(device if device is not None else "cuda")
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        n = len(cfgs)
        arr = (Config * n)(*cfgs)
        nbytes = c_uint64()
        check(self._lib.cnlos_batch_workspace_bytes(arr, n, byref(nbytes)))
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        self._masks = [np.ascontiguousarray(m, dtype=np.uint8) for m in masks]
        for c, m in zip(cfgs, self._masks):
            if m.shape != (c.nx, c.ny):
                raise ValueError(f"mask must be {(c.nx, c.ny)}")
        mp = (POINTER(c_uint8) * n)(*[m.ctypes.data_as(POINTER(c_uint8)) for m in self._masks])
        h = c_void_p()
        with torch.cuda.device(self.device):
            st = self._lib.cnlos_batch_create(arr, n, mp, c_void_p(self.workspace.data_ptr()),
                                              nbytes, c_void_p(self.stream.cuda_stream), byref(h))
        self._h = h
        if st != OK:
            msg = last_error()
            self.close()
            raise CnlosError(st, msg)
        self.members = []
        for i in range(n):
            mh = c_void_p()
            check(self._lib.cnlos_batch_member(self._h, i, byref(mh)))
            self.members.append(Problem(cfgs[i], self._masks[i], _member=(mh, self)))

    def __len__(self):
        return len(self.members)

    def run(self, iters=0):
        """Advance every member; returns (status, [report dict per member])."""
        n = len(self.members)
        reps = (Report * n)()
        st = self._lib.cnlos_batch_run(self._h, int(iters), reps)
        return st, [_report_dict(r) for r in reps]

    def close(self):
        if self._h is not None and self._h.value is not None:
            for m in getattr(self, "members", []):
                m._h = None
            self._lib.cnlos_batch_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_many(batches, iters=0):
    """Advance several batches at once (each on its own stream, overlapping on
    the device); returns (status, [[report dict per member] per batch])."""
    lib = load()
    k = len(batches)
    hs = (c_void_p * k)(*[b._h for b in batches])
    arrs = [(Report * len(b.members))() for b in batches]
    ptrs = (POINTER(Report) * k)(*[ctypes.cast(a, POINTER(Report)) for a in arrs])
    st = lib.cnlos_batch_run_many(hs, k, int(iters), ptrs)
    return st, [[_report_dict(r) for r in a] for a in arrs]


class Server:
    """Continuous-batching request loop of the library: requests of any
    supported shape are admitted into slot groups of their shape as slots and
    arena memory free up; every step advances all groups, each on its own
    stream.  The arena (HBM budget) is one device allocation made here."""

    def __init__(self, arena_bytes, slots=8, rounds=8, device=None):
        import torch
        self._lib = load()
        self._h = None
        self.device = torch.device(device if device is not None else "cuda")
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=self.device)
        self._keep = {}
        h = c_void_p()
        check(self._lib.cnlos_server_create(c_void_p(self.arena.data_ptr()), c_uint64(self.arena.numel()),
                                            int(slots), int(rounds), byref(h)))
        self._h = h

    def submit(self, cfg, mask, tau0, out, rid):
        """Queue a request; tau0 and out (device float32 [nx][ny][nt]) are kept
        alive here until the request completes."""
        m = np.ascontiguousarray(mask, dtype=np.uint8)
        req = Request()
        req.cfg = cfg
        req.mask_host = m.ctypes.data_as(POINTER(c_uint8))
        req.tau0_dev = c_void_p(tau0.data_ptr())
        req.out_dev = c_void_p(out.data_ptr())
        req.id = int(rid)
        check(self._lib.cnlos_server_submit(self._h, byref(req)))
        self._keep[int(rid)] = (tau0, out)

    def step(self):
        a, q = c_int32(), c_int32()
        check(self._lib.cnlos_server_step(self._h, byref(a), byref(q)))
        return a.value, q.value

    def poll(self, cap=1024):
        buf = (Completion * cap)()
        n = c_int32()
        check(self._lib.cnlos_server_poll(self._h, buf, cap, byref(n)))
        out = []
        for i in range(n.value):
            c = buf[i]
            out.append({f: getattr(c, f) for f, _ in Completion._fields_})
            self._keep.pop(int(c.id), None)
        return out

    def fail_next_groups(self, count):
        """Testing hook: the next ``count`` slot-group creations fail."""
        check(self._lib.cnlos_server_fail_next_groups(self._h, int(count)))

    def usage(self):
        b, g = c_uint64(), c_int32()
        check(self._lib.cnlos_server_usage(self._h, byref(b), byref(g)))
        return int(b.value), int(g.value)

    def close(self):
        if self._h is not None and self._h.value is not None:
            self._lib.cnlos_server_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
