"""Thin ctypes binding of libigmres.so (C-ABI in include/igmres.h).

Argument marshalling only: every step of the method runs in the HIP library.
PyTorch supplies device memory and the current HIP stream.  Importing this
module loads the library and raises ImportError if it has not been built --
there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("IGMRES_LIB") or os.path.join(HERE, "libigmres.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2211_04299_amd.build`")
_lib = C.CDLL(LIB_PATH)

# ---- enums (include/igmres.h) ---------------------------------------------
IG_OK, IG_E_INVALID, IG_E_NOMEM, IG_E_DEVICE, IG_E_NOCONV, IG_E_NUMERIC, IG_E_TOO_LARGE = (
    0, -1, -2, -3, -4, -5, -6)
STATUS_NAMES = {0: "IG_OK", -1: "IG_E_INVALID", -2: "IG_E_NOMEM", -3: "IG_E_DEVICE",
                -4: "IG_E_NOCONV", -5: "IG_E_NUMERIC", -6: "IG_E_TOO_LARGE"}
IG_FMT_CSR, IG_FMT_DENSE = 0, 1
IG_FP64, IG_FP32, IG_BF16 = 0, 1, 2
DTYPES = {"fp64": IG_FP64, "fp32": IG_FP32, "bf16": IG_BF16}
IG_MODE_FP64, IG_MODE_MIXED = 0, 1
IG_MAX_RESTART = 128
IG_NOALLOC_SCRATCH_BYTES = 32 << 20
ENGINE_AUTO, ENGINE_STREAM, ENGINE_PERSISTENT = 0, 1, 2
IG_PROFILE_CLASSES = 8
PROFILE_CLASS_NAMES = ["bellman", "japply", "gram_schmidt", "update", "residual", "vi_sweep", "other",
                       "persistent"]

EXPORTS = ["ig_params_default", "mdp_create", "mdp_destroy", "mdp_get_info", "bellman_apply",
           "policy_eval_gmres", "igmres_pi_solve", "pi_solve", "opi_solve", "ipi_vi_solve",
           "igmres_pi_solve_noalloc", "ig_profile_enable", "ig_profile_sample", "ig_profile_read",
           "ig_last_error", "ig_server_config_default",
           "srv_create", "srv_submit", "srv_poll", "srv_result", "srv_get_info", "srv_destroy"]


class MdpDesc(C.Structure):
    _fields_ = [("n", C.c_int64), ("m", C.c_int32), ("gamma", C.c_double), ("fmt", C.c_int),
                ("row_ptr", C.c_void_p), ("col", C.c_void_p), ("val", C.c_void_p),
                ("val_type", C.c_int), ("cost", C.c_void_p), ("store", C.c_int),
                ("inputs_on_device", C.c_int32), ("validate", C.c_int32),
                ("admissible", C.c_void_p), ("refine", C.c_int32)]


class Params(C.Structure):
    _fields_ = [("alpha", C.c_double), ("restart", C.c_int32), ("max_outer", C.c_int32),
                ("max_inner", C.c_int32), ("tol", C.c_double), ("mode", C.c_int),
                ("opi_sweeps", C.c_int32), ("forcing", C.c_int32), ("eval_rtol", C.c_double),
                ("engine", C.c_int32), ("blocks", C.c_int32), ("precond", C.c_int32),
                ("polish", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("outer", C.c_int32), ("inner", C.c_int32), ("restarts", C.c_int32),
                ("bellman_passes", C.c_int32), ("explicit_residuals", C.c_int32),
                ("breakdowns", C.c_int32), ("stagnations", C.c_int32), ("converged", C.c_int32),
                ("res_inf", C.c_double), ("cert_bound", C.c_double), ("time_ms", C.c_double),
                ("alg_bytes", C.c_double), ("latency_ms", C.c_double), ("queue_ms", C.c_double),
                ("prep_ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class MdpInfo(C.Structure):
    _fields_ = [("n", C.c_int64), ("m", C.c_int32), ("max_width", C.c_int32), ("nnz", C.c_int64),
                ("stored_entries", C.c_int64), ("p_bytes", C.c_int64), ("store", C.c_int),
                ("fmt", C.c_int), ("gamma", C.c_double), ("persistent_ok", C.c_int32),
                ("persistent_blocks", C.c_int32), ("refine", C.c_int32), ("inner_p_bytes", C.c_int64)]


class ServerConfig(C.Structure):
    _fields_ = [("device", C.c_int32), ("slots", C.c_int32), ("prep_threads", C.c_int32),
                ("block_slices", C.c_int32), ("max_states", C.c_int64), ("hbm_budget", C.c_size_t)]


class ServerInfo(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("failed", C.c_int64),
                ("queued", C.c_int32), ("preparing", C.c_int32), ("ready", C.c_int32),
                ("running", C.c_int32), ("peak_running", C.c_int32), ("xcd_units_cap", C.c_int32),
                ("arena_bytes", C.c_size_t), ("arena_used", C.c_size_t), ("arena_peak", C.c_size_t)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_P = C.c_void_p
_sig = {
    "ig_params_default": (None, [C.POINTER(Params), C.c_double]),
    "mdp_create": (C.c_int, [C.POINTER(MdpDesc), _P, C.POINTER(_P)]),
    "mdp_destroy": (None, [_P]),
    "mdp_get_info": (C.c_int, [_P, C.POINTER(MdpInfo)]),
    "bellman_apply": (C.c_int, [_P, _P, _P, _P, _P, _P]),
    "policy_eval_gmres": (C.c_int, [_P, _P, _P, C.POINTER(Params), C.POINTER(Stats), _P]),
    "igmres_pi_solve": (C.c_int, [_P, _P, _P, C.POINTER(Params), C.POINTER(Stats), _P]),
    "igmres_pi_solve_noalloc": (C.c_int, [_P, _P, _P, C.POINTER(Params), C.POINTER(Stats), _P]),
    "pi_solve": (C.c_int, [_P, _P, _P, C.POINTER(Params), C.POINTER(Stats), _P]),
    "opi_solve": (C.c_int, [_P, _P, _P, C.POINTER(Params), C.POINTER(Stats), _P]),
    "ipi_vi_solve": (C.c_int, [_P, _P, _P, C.POINTER(Params), C.POINTER(Stats), _P]),
    "ig_profile_enable": (C.c_int, [_P, C.c_uint]),
    "ig_profile_sample": (C.c_int, [_P, C.c_int]),
    "ig_profile_read": (C.c_int, [_P, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.c_int]),
    "ig_last_error": (C.c_char_p, []),
    "ig_server_config_default": (None, [C.POINTER(ServerConfig)]),
    "srv_create": (C.c_int, [C.POINTER(ServerConfig), C.POINTER(_P)]),
    "srv_submit": (C.c_int, [_P, C.POINTER(MdpDesc), _P, C.POINTER(Params), C.POINTER(C.c_uint64)]),
    "srv_poll": (C.c_int, [_P, C.c_uint64, C.POINTER(C.c_int32)]),
    "srv_result": (C.c_int, [_P, C.c_uint64, _P, _P, C.POINTER(Stats)]),
    "srv_get_info": (C.c_int, [_P, C.POINTER(ServerInfo)]),
    "srv_destroy": (None, [_P]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class IgError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = _lib.ig_last_error().decode()
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")


def _check(status, where, ok=(IG_OK,)):
    if status not in ok:
        raise IgError(status, where)
    return status


def last_error() -> str:
    return _lib.ig_last_error().decode()


def params_default(gamma: float, **kw) -> Params:
    p = Params()
    _lib.ig_params_default(C.byref(p), float(gamma))
    for k, v in kw.items():
        if k == "mode" and isinstance(v, str):
            v = IG_MODE_MIXED if v == "mixed" else IG_MODE_FP64
        setattr(p, k, v)
    return p


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    return x.data_ptr()  # torch tensor


def _stream(stream):
    if stream is not None:
        return stream
    import torch
    return torch.cuda.current_stream().cuda_stream


class Mdp:
    """Owns one device-resident MDP (an ig_mdp_t)."""

    def __init__(self, handle, n, m, gamma):
        self.handle = handle
        self.n, self.m, self.gamma = n, m, gamma

    def close(self):
        if self.handle:
            _lib.mdp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def info(self) -> MdpInfo:
        inf = MdpInfo()
        _check(_lib.mdp_get_info(self.handle, C.byref(inf)), "mdp_get_info")
        return inf

    # ---- entry points -----------------------------------------------------
    def bellman_apply(self, V, TV=None, pi=None, res_inf=None, stream=None):
        _check(_lib.bellman_apply(self.handle, _ptr(V), _ptr(TV), _ptr(pi), _ptr(res_inf),
                                  _stream(stream)), "bellman_apply")

    def _solve(self, fn, name, V, pi, params, stream, allow_noconv):
        st = Stats()
        rc = fn(self.handle, _ptr(V), _ptr(pi), C.byref(params), C.byref(st), _stream(stream))
        _check(rc, name, (IG_OK, IG_E_NOCONV) if allow_noconv else (IG_OK,))
        d = st.as_dict()
        d["status"] = rc
        return d

    def policy_eval_gmres(self, pi, V, params, stream=None, allow_noconv=False):
        st = Stats()
        rc = _lib.policy_eval_gmres(self.handle, _ptr(pi), _ptr(V), C.byref(params), C.byref(st),
                                    _stream(stream))
        _check(rc, "policy_eval_gmres", (IG_OK, IG_E_NOCONV) if allow_noconv else (IG_OK,))
        d = st.as_dict()
        d["status"] = rc
        return d

    def igmres_pi_solve(self, V, pi, params, stream=None, allow_noconv=False):
        return self._solve(_lib.igmres_pi_solve, "igmres_pi_solve", V, pi, params, stream, allow_noconv)

    def igmres_pi_solve_noalloc(self, V, pi, params, stream=None, allow_noconv=False):
        return self._solve(_lib.igmres_pi_solve_noalloc, "igmres_pi_solve_noalloc", V, pi, params,
                           stream, allow_noconv)

    def pi_solve(self, V, pi, params, stream=None, allow_noconv=False):
        return self._solve(_lib.pi_solve, "pi_solve", V, pi, params, stream, allow_noconv)

    def opi_solve(self, V, pi, params, stream=None, allow_noconv=False):
        return self._solve(_lib.opi_solve, "opi_solve", V, pi, params, stream, allow_noconv)

    def ipi_vi_solve(self, V, pi, params, stream=None, allow_noconv=False):
        return self._solve(_lib.ipi_vi_solve, "ipi_vi_solve", V, pi, params, stream, allow_noconv)

    # ---- measurement ------------------------------------------------------
    def profile_enable(self, mask: int):
        _check(_lib.ig_profile_enable(self.handle, mask), "ig_profile_enable")

    def profile_sample(self, every: int):
        _check(_lib.ig_profile_sample(self.handle, int(every)), "ig_profile_sample")

    def profile_read(self, reset=True):
        ms = (C.c_double * IG_PROFILE_CLASSES)()
        cnt = (C.c_int64 * IG_PROFILE_CLASSES)()
        _check(_lib.ig_profile_read(self.handle, ms, cnt, int(reset)), "ig_profile_read")
        return {PROFILE_CLASS_NAMES[k]: (ms[k], cnt[k]) for k in range(IG_PROFILE_CLASSES)}


def _desc(mdp, store, validate, refine=False):
    """MdpDesc for a synth.MDP-like object with host arrays, plus the arrays
    it points into (to be kept alive by the caller)."""
    d = MdpDesc()
    d.refine = int(refine)
    d.n, d.m, d.gamma = mdp.n, mdp.m, float(mdp.gamma)
    keep = []
    if mdp.fmt == "csr":
        d.fmt = IG_FMT_CSR
        rp = np.ascontiguousarray(mdp.row_ptr, dtype=np.int64)
        col = np.ascontiguousarray(mdp.col, dtype=np.int32)
        val = np.ascontiguousarray(mdp.val)
        keep += [rp, col, val]
        d.row_ptr, d.col, d.val = rp.ctypes.data, col.ctypes.data, val.ctypes.data
    else:
        d.fmt = IG_FMT_DENSE
        val = np.ascontiguousarray(mdp.P)
        keep.append(val)
        d.val = val.ctypes.data
    d.val_type = {np.dtype(np.float64): IG_FP64, np.dtype(np.float32): IG_FP32,
                  np.dtype(np.uint16): IG_BF16}[val.dtype]
    cost = np.ascontiguousarray(mdp.cost, dtype=np.float64)
    keep.append(cost)
    d.cost = cost.ctypes.data
    d.store = DTYPES[store]
    d.inputs_on_device = 0
    d.validate = int(validate)
    adm = getattr(mdp, "adm", None)
    if adm is not None:  # action sets A(s): admissible[s*m + a]
        a8 = np.ascontiguousarray(np.asarray(adm).reshape(-1), dtype=np.uint8)
        if a8.size != mdp.n * mdp.m:
            raise ValueError("adm must hold n*m entries")
        keep.append(a8)
        d.admissible = a8.ctypes.data
    return d, keep


def _desc_device(mdp, store, validate, refine=False):
    """Description of a CSR MDP whose arrays are device tensors (row_ptr
    int64, col int32, val float64/float32/int16-or-uint16 bf16 patterns,
    cost float64, adm uint8/bool or None)."""
    import torch
    if mdp.fmt != "csr":
        raise ValueError("device inputs are taken for CSR MDPs")
    d = MdpDesc()
    d.refine = int(refine)
    d.n, d.m, d.gamma = mdp.n, mdp.m, float(mdp.gamma)
    d.fmt = IG_FMT_CSR
    vt = {torch.float64: IG_FP64, torch.float32: IG_FP32, torch.int16: IG_BF16,
          torch.uint16: IG_BF16, torch.bfloat16: IG_BF16}[mdp.val.dtype]
    for name, t, dt in (("row_ptr", mdp.row_ptr, torch.int64), ("col", mdp.col, torch.int32),
                        ("cost", mdp.cost, torch.float64)):
        if t.dtype != dt or not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous device tensor of {dt}")
    d.row_ptr, d.col, d.val, d.cost = (mdp.row_ptr.data_ptr(), mdp.col.data_ptr(),
                                       mdp.val.data_ptr(), mdp.cost.data_ptr())
    d.val_type = vt
    d.store = DTYPES[store]
    d.inputs_on_device = 1
    d.validate = int(validate)
    adm = getattr(mdp, "adm", None)
    if adm is not None:
        d.admissible = adm.data_ptr()
    return d, [mdp]


def mdp_create(mdp, store: str = "fp64", validate: bool = True, stream=None,
               inputs_on_device: bool = False, refine: bool = False) -> Mdp:
    """Create a device MDP from a synth.MDP-like object with host arrays
    (fmt "csr": row_ptr/col/val; "dense": P).  `mdp.val` / `mdp.P` may be
    float64, float32 or uint16 (bf16 bit patterns).  inputs_on_device: the
    CSR arrays, costs and mask are device tensors instead.  refine (with
    store "bf16"): BF16 products inside GMRES beside an FP32 copy for every
    other pass (ig_mdp_desc.refine)."""
    d, keep = (_desc_device if inputs_on_device else _desc)(mdp, store, validate, refine)
    h = C.c_void_p()
    _check(_lib.mdp_create(C.byref(d), stream, C.byref(h)), "mdp_create")
    del keep
    return Mdp(h, mdp.n, mdp.m, float(mdp.gamma))


def server_config_default(**kw) -> ServerConfig:
    c = ServerConfig()
    _lib.ig_server_config_default(C.byref(c))
    for k, v in kw.items():
        setattr(c, k, v)
    return c


class Server:
    """Continuous-batching solver service (an ig_server_t).  submit() returns
    a ticket at once; the request's host arrays are held here until result()
    collects it (the library borrows them)."""

    def __init__(self, config: ServerConfig | None = None, **kw):
        cfg = config if config is not None else server_config_default(**kw)
        h = C.c_void_p()
        _check(_lib.srv_create(C.byref(cfg), C.byref(h)), "srv_create")
        self.handle = h
        self.config = cfg
        self._held = {}

    def submit(self, mdp, params: Params, store: str = "fp32", validate: bool = True, V0=None) -> int:
        d, keep = _desc(mdp, store, validate)
        v0 = None
        if V0 is not None:
            v0 = np.ascontiguousarray(V0, dtype=np.float64)
            keep.append(v0)
        t = C.c_uint64()
        _check(_lib.srv_submit(self.handle, C.byref(d), _ptr(v0), C.byref(params), C.byref(t)),
               "srv_submit")
        self._held[t.value] = (keep, mdp.n)
        return t.value

    def poll(self, ticket: int) -> bool:
        done = C.c_int32()
        _check(_lib.srv_poll(self.handle, ticket, C.byref(done)), "srv_poll")
        return bool(done.value)

    def result(self, ticket: int, allow_noconv: bool = False):
        """Wait for the ticket; returns (V float64[n], pi int32[n], stats dict)."""
        _, n = self._held[ticket]
        V = np.zeros(n, np.float64)
        pi = np.zeros(n, np.int32)
        st = Stats()
        rc = _lib.srv_result(self.handle, ticket, V.ctypes.data, pi.ctypes.data, C.byref(st))
        self._held.pop(ticket, None)
        _check(rc, "srv_result", (IG_OK, IG_E_NOCONV) if allow_noconv else (IG_OK,))
        d = st.as_dict()
        d["status"] = rc
        return V, pi, d

    def info(self) -> dict:
        inf = ServerInfo()
        _check(_lib.srv_get_info(self.handle, C.byref(inf)), "srv_get_info")
        return inf.as_dict()

    def close(self):
        if self.handle:
            _lib.srv_destroy(self.handle)
            self.handle = None
            self._held.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
