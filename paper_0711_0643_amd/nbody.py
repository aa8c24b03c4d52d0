"""ctypes binding of libnbody (argument marshalling only).

Every step of the integration runs in the HIP library; this module checks
shapes and dtypes, allocates the workspace as a torch tensor on the GPU,
and passes raw pointers and the current torch stream to the C ABI.  There is
no CPU fallback: without the built library every entry point raises.
"""
from __future__ import annotations

import ctypes
import math
from pathlib import Path

import numpy as np

_PKG = Path(__file__).resolve().parent
_LIB_PATH = _PKG / "libnbody.so"

FP64 = 0
MIXED = 1

# nbody_status codes (include/nbody.h)
NBODY_OK = 0
NBODY_E_INVAL = -1
NBODY_E_NOMEM = -2
NBODY_E_HIP = -3
NBODY_E_STATE = -4
NBODY_E_DTMIN = -5
NBODY_E_NONFINITE = -6
NBODY_E_INDEX = -7
_STATUS = {code: name for name, code in list(globals().items()) if name.startswith("NBODY_")}

EXPORTED = [
    "nbody_default_params",
    "nbody_workspace_bytes",
    "nbody_init",
    "nbody_set_params",
    "nbody_predict",
    "nbody_force",
    "nbody_force_noalloc",
    "nbody_perturbers",
    "nbody_correct",
    "nbody_step",
    "nbody_sync",
    "nbody_energy",
    "nbody_diagnostics",
    "nbody_progress",
    "nbody_state_bytes",
    "nbody_get_state",
    "nbody_set_state",
    "nbody_get_layout",
    "nbody_get_tuning",
    "nbody_set_tuning",
    "nbody_profile_force",
    "nbody_profile_read",
    "nbody_destroy",
    "nbody_strerror",
]


def status_name(code: int) -> str:
    return _STATUS.get(code, f"status {code}")


class NBodyError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {status_name(code)}")


class Params(ctypes.Structure):
    _fields_ = [
        ("eta", ctypes.c_double),
        ("eta_init", ctypes.c_double),
        ("dt_max", ctypes.c_double),
        ("dt_min", ctypes.c_double),
        ("precision", ctypes.c_int32),
        ("compute_pot", ctypes.c_int32),
    ]


class Layout(ctypes.Structure):
    _fields_ = [
        ("n_total", ctypes.c_int64),
        ("n_clusters", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("m", ctypes.c_size_t),
        ("x", ctypes.c_size_t),
        ("v", ctypes.c_size_t),
        ("a", ctypes.c_size_t),
        ("k", ctypes.c_size_t),
        ("t", ctypes.c_size_t),
        ("dt", ctypes.c_size_t),
        ("xp", ctypes.c_size_t),
        ("vp", ctypes.c_size_t),
        ("pot", ctypes.c_size_t),
        ("order", ctypes.c_size_t),
    ]


class Tuning(ctypes.Structure):
    _fields_ = [
        ("target_items", ctypes.c_int32),
        ("min_block", ctypes.c_int32 * 4),
        ("grid", ctypes.c_int32),
        ("mixed_format", ctypes.c_int32),
        ("rsq_bias_correct", ctypes.c_int32),
        ("near_tau", ctypes.c_double),
        ("small_cluster_n", ctypes.c_int32),
        ("small_min_block", ctypes.c_int32 * 4),
        ("near_tau_k", ctypes.c_double),
        ("mid_tau", ctypes.c_double),
        ("window", ctypes.c_int32),
        ("waves", ctypes.c_int32),
        ("tile", ctypes.c_int32),
        ("pred_in_force", ctypes.c_int32),
    ]


_lib = None


def library_path() -> Path:
    return _LIB_PATH


def lib() -> ctypes.CDLL:
    """Load libnbody.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        # torch ships its own HIP runtime; load it first so that libnbody binds
        # to the same runtime instance (one HIP runtime per process).
        import torch  # noqa: F401

        if not _LIB_PATH.exists():
            raise RuntimeError(f"{_LIB_PATH} is not built; run paper_0711_0643_amd/build.py")
        L = ctypes.CDLL(str(_LIB_PATH))
        p, i32, i64, f64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
        st = ctypes.c_int
        L.nbody_default_params.argtypes = [ctypes.POINTER(Params)]
        L.nbody_default_params.restype = None
        L.nbody_workspace_bytes.argtypes = [i64, i32, ctypes.POINTER(Params), ctypes.POINTER(sz)]
        L.nbody_workspace_bytes.restype = st
        L.nbody_init.argtypes = [ctypes.POINTER(p), i64, i32, p, p, p, p, p, ctypes.POINTER(Params), p, sz, p]
        L.nbody_init.restype = st
        L.nbody_set_params.argtypes = [p, ctypes.POINTER(Params)]
        L.nbody_set_params.restype = st
        L.nbody_predict.argtypes = [p, p]
        L.nbody_predict.restype = st
        L.nbody_force.argtypes = [p, p, p, i64, p, p, p]
        L.nbody_force.restype = st
        L.nbody_force_noalloc.argtypes = [p, p, p, i64, p, p, p]
        L.nbody_force_noalloc.restype = st
        L.nbody_perturbers.argtypes = [p, p, p, i64, p, ctypes.c_int32, p, p]
        L.nbody_perturbers.restype = st
        L.nbody_correct.argtypes = [p, p, p, i64, p, p]
        L.nbody_correct.restype = st
        L.nbody_step.argtypes = [p, i32, f64]
        L.nbody_step.restype = st
        L.nbody_sync.argtypes = [p]
        L.nbody_sync.restype = st
        L.nbody_energy.argtypes = [p, p]
        L.nbody_energy.restype = st
        L.nbody_diagnostics.argtypes = [p, p]
        L.nbody_diagnostics.restype = st
        L.nbody_progress.argtypes = [p, p, p, p]
        L.nbody_progress.restype = st
        L.nbody_state_bytes.argtypes = [p, ctypes.POINTER(sz)]
        L.nbody_state_bytes.restype = st
        L.nbody_get_state.argtypes = [p, p, sz]
        L.nbody_get_state.restype = st
        L.nbody_set_state.argtypes = [p, p, sz]
        L.nbody_set_state.restype = st
        L.nbody_get_layout.argtypes = [p, ctypes.POINTER(Layout)]
        L.nbody_get_layout.restype = st
        L.nbody_get_tuning.argtypes = [p, ctypes.POINTER(Tuning)]
        L.nbody_get_tuning.restype = st
        L.nbody_set_tuning.argtypes = [p, ctypes.POINTER(Tuning)]
        L.nbody_set_tuning.restype = st
        L.nbody_profile_force.argtypes = [p, i32]
        L.nbody_profile_force.restype = st
        L.nbody_profile_read.argtypes = [p, ctypes.POINTER(f64), ctypes.POINTER(i64)]
        L.nbody_profile_read.restype = st
        L.nbody_destroy.argtypes = [p]
        L.nbody_destroy.restype = st
        L.nbody_strerror.argtypes = [st]
        L.nbody_strerror.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(code: int, what: str) -> None:
    if code != 0:
        raise NBodyError(code, what)


def default_params(**kw) -> Params:
    p = Params()
    lib().nbody_default_params(ctypes.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise TypeError(f"unknown parameter {k}")
        setattr(p, k, v)
    return p


def _f64_host(a, shape) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


class Sim:
    """One or more independent clusters on one GPU.

    ``m`` (N,), ``x``/``v`` (3, N) host arrays (float64, structure-of-arrays);
    ``cluster_offsets`` (n_clusters+1,) int64 with [0] = 0 and [-1] = N
    (default: one cluster); ``eps`` scalar or (n_clusters,).
    """

    def __init__(self, m, x, v, eps, cluster_offsets=None, precision: int = FP64, eta: float = 0.01,
                 eta_init: float = 0.01, dt_max: float = 0.125, dt_min: float = 2.0**-40,
                 compute_pot: bool = False, device: str = "cuda:0", stream=None):
        import torch

        self._torch = torch
        m = np.ascontiguousarray(np.asarray(m, dtype=np.float64))
        n = m.shape[0]
        x = _f64_host(x, (3, n))
        v = _f64_host(v, (3, n))
        if cluster_offsets is None:
            cluster_offsets = [0, n]
        coff = np.ascontiguousarray(np.asarray(cluster_offsets, dtype=np.int64))
        nc = coff.shape[0] - 1
        eps_arr = np.ascontiguousarray(np.broadcast_to(np.asarray(eps, dtype=np.float64), (nc,)).copy())
        self.n, self.nc = n, nc
        self.device = torch.device(device)
        self.params = default_params(eta=eta, eta_init=eta_init, dt_max=dt_max, dt_min=dt_min,
                                     precision=int(precision), compute_pot=int(bool(compute_pot)))
        nbytes = ctypes.c_size_t(0)
        _check(lib().nbody_workspace_bytes(n, nc, ctypes.byref(self.params), ctypes.byref(nbytes)),
               "nbody_workspace_bytes")
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._ctx = ctypes.c_void_p(None)
        _check(lib().nbody_init(ctypes.byref(self._ctx), n, nc, coff.ctypes.data, m.ctypes.data, x.ctypes.data,
                                v.ctypes.data, eps_arr.ctypes.data, ctypes.byref(self.params),
                                self.workspace.data_ptr(), int(nbytes.value), self.stream.cuda_stream),
               "nbody_init")
        self.cluster_offsets = coff
        self.eps = eps_arr
        lay = Layout()
        _check(lib().nbody_get_layout(self._ctx, ctypes.byref(lay)), "nbody_get_layout")
        self._layout = lay

    # -- the state inside the workspace ---------------------------------------------
    # The library stores particles in its own order (Morton order inside each
    # cluster); slot q holds particle order[q].  The properties below return
    # the state in particle-id order (gathered copies); ``raw`` views give the
    # arrays in storage order without a copy.
    @property
    def order(self):
        """(N,) int64 tensor: the particle id stored at each slot."""
        off = self._layout.order
        return self.workspace[off: off + 4 * self.n].view(self._torch.int32).long()

    @property
    def slot_of(self):
        """(N,) int64 tensor: the slot of each particle id."""
        o = self.order
        inv = self._torch.empty_like(o)
        inv[o] = self._torch.arange(self.n, device=o.device)
        return inv

    def raw(self, name: str):
        """View of a state array (m, x, v, a, k, t, dt, xp, vp) in storage order."""
        rows = 3 if name in ("x", "v", "a", "k", "xp", "vp") else 1
        off = getattr(self._layout, name)
        t = self.workspace[off: off + 8 * rows * self.n].view(self._torch.float64)
        return t.view(rows, self.n) if rows > 1 else t

    def _view(self, off: int, rows: int):
        t = self.workspace[off: off + 8 * rows * self.n].view(self._torch.float64)
        t = t.view(rows, self.n) if rows > 1 else t
        return t[..., self.slot_of]

    def storage_active(self, n_act=None):
        """Particle ids of the first n_act slots of a single cluster (all by
        default): an active list in storage order, the fastest for the mixed
        force pass."""
        o = self.order.to(self._torch.int32)
        return o if n_act is None else o[:n_act]

    @property
    def x(self):
        return self._view(self._layout.x, 3)

    @property
    def v(self):
        return self._view(self._layout.v, 3)

    @property
    def a(self):
        return self._view(self._layout.a, 3)

    @property
    def k(self):
        return self._view(self._layout.k, 3)

    @property
    def t(self):
        return self._view(self._layout.t, 1)

    @property
    def dt(self):
        return self._view(self._layout.dt, 1)

    @property
    def xp(self):
        return self._view(self._layout.xp, 3)

    @property
    def vp(self):
        return self._view(self._layout.vp, 3)

    @property
    def m(self):
        return self._view(self._layout.m, 1)

    # -- calls -----------------------------------------------------------------------
    def set_precision(self, precision: int) -> None:
        self.params.precision = int(precision)
        _check(lib().nbody_set_params(self._ctx, ctypes.byref(self.params)), "nbody_set_params")

    def set_params(self, **kw) -> None:
        for k, v in kw.items():
            setattr(self.params, k, v)
        _check(lib().nbody_set_params(self._ctx, ctypes.byref(self.params)), "nbody_set_params")

    def get_tuning(self) -> dict:
        t = Tuning()
        _check(lib().nbody_get_tuning(self._ctx, ctypes.byref(t)), "nbody_get_tuning")
        return {"target_items": t.target_items, "min_block": list(t.min_block), "grid": t.grid,
                "mixed_format": t.mixed_format, "rsq_bias_correct": t.rsq_bias_correct,
                "near_tau": t.near_tau, "small_cluster_n": t.small_cluster_n,
                "small_min_block": list(t.small_min_block), "near_tau_k": t.near_tau_k,
                "mid_tau": t.mid_tau, "window": t.window, "waves": t.waves, "tile": t.tile,
                "pred_in_force": t.pred_in_force}

    def set_tuning(self, **kw) -> None:
        cur = self.get_tuning()
        cur.update(kw)
        t = Tuning()
        t.target_items = int(cur["target_items"])
        for i in range(4):
            t.min_block[i] = int(cur["min_block"][i])
        t.grid = int(cur["grid"])
        t.mixed_format = int(cur["mixed_format"])
        t.rsq_bias_correct = int(cur["rsq_bias_correct"])
        t.near_tau = float(cur["near_tau"])
        t.near_tau_k = float(cur["near_tau_k"])
        t.mid_tau = float(cur["mid_tau"])
        t.window = int(cur["window"])
        t.waves = int(cur["waves"])
        t.tile = int(cur["tile"])
        t.pred_in_force = int(cur["pred_in_force"])
        t.small_cluster_n = int(cur["small_cluster_n"])
        for i in range(4):
            t.small_min_block[i] = int(cur["small_min_block"][i])
        _check(lib().nbody_set_tuning(self._ctx, ctypes.byref(t)), "nbody_set_tuning")

    def profile_force(self, enable: bool = True) -> None:
        _check(lib().nbody_profile_force(self._ctx, int(bool(enable))), "nbody_profile_force")

    def profile_read(self):
        """(summed force-kernel milliseconds, launches) since the last read."""
        ms = ctypes.c_double(0.0)
        n = ctypes.c_int64(0)
        _check(lib().nbody_profile_read(self._ctx, ctypes.byref(ms), ctypes.byref(n)), "nbody_profile_read")
        return ms.value, n.value

    def predict(self, t_pred=None) -> None:
        if t_pred is None:
            _check(lib().nbody_predict(self._ctx, None), "nbody_predict")
        else:
            tp = np.ascontiguousarray(np.broadcast_to(np.asarray(t_pred, dtype=np.float64), (self.nc,)).copy())
            _check(lib().nbody_predict(self._ctx, tp.ctypes.data), "nbody_predict")

    def _active(self, active_idx, active_offsets):
        torch = self._torch
        act = torch.as_tensor(active_idx, dtype=torch.int32, device=self.device).contiguous()
        if active_offsets is None:
            if self.nc != 1:
                raise ValueError("active_offsets is required with several clusters")
            active_offsets = [0, act.numel()]
        aoff = torch.as_tensor(active_offsets, dtype=torch.int64, device=self.device).contiguous()
        if aoff.numel() != self.nc + 1:
            raise ValueError("active_offsets must have n_clusters + 1 entries")
        return act, aoff

    def force(self, active_idx, active_offsets=None, pot: bool = False, out=None):
        """a, k (3, n_act) and phi (n_act,) float64 tensors on the device."""
        return self._force("nbody_force", active_idx, active_offsets, pot, out)

    def force_noalloc(self, active_idx, active_offsets=None, pot: bool = False, out=None):
        """As force(), through nbody_force_noalloc (partials in the library's
        static device scratch)."""
        return self._force("nbody_force_noalloc", active_idx, active_offsets, pot, out)

    def _force(self, entry, active_idx, active_offsets, pot, out):
        torch = self._torch
        act, aoff = self._active(active_idx, active_offsets)
        na = act.numel()
        if out is None:
            acc = torch.empty((3, na), dtype=torch.float64, device=self.device)
            jerk = torch.empty((3, na), dtype=torch.float64, device=self.device)
            ph = torch.empty((na,), dtype=torch.float64, device=self.device) if pot else None
        else:
            acc, jerk, ph = out
        _check(getattr(lib(), entry)(self._ctx, act.data_ptr(), aoff.data_ptr(), na, acc.data_ptr(), jerk.data_ptr(),
                                     ph.data_ptr() if ph is not None else None), entry)
        self._keep = (act, aoff)  # alive until the stream has consumed them
        return acc, jerk, ph

    def perturbers(self, active_idx, threshold, active_offsets=None, max_pert: int = 256):
        """Perturber lists (nbody_perturbers): threshold per cluster (sequence
        or tensor of n_clusters floats); returns lists (n_act, max_pert) and
        counts (n_act,) int32 tensors on the device."""
        torch = self._torch
        act, aoff = self._active(active_idx, active_offsets)
        na = act.numel()
        thr = torch.as_tensor(threshold, dtype=torch.float64).reshape(-1).to(self.device).contiguous()
        if thr.numel() != self.nc:
            raise ValueError("threshold needs one value per cluster")
        lists = torch.empty((na, max_pert), dtype=torch.int32, device=self.device)
        counts = torch.empty((na,), dtype=torch.int32, device=self.device)
        _check(lib().nbody_perturbers(self._ctx, act.data_ptr(), aoff.data_ptr(), na, thr.data_ptr(), int(max_pert),
                                      lists.data_ptr(), counts.data_ptr()), "nbody_perturbers")
        self._keep = (act, aoff, thr)  # alive until the stream has consumed them
        return lists, counts

    def correct(self, active_idx, acc, jerk, active_offsets=None) -> None:
        act, aoff = self._active(active_idx, active_offsets)
        na = act.numel()
        acc = acc.contiguous()
        jerk = jerk.contiguous()
        if tuple(acc.shape) != (3, na) or tuple(jerk.shape) != (3, na):
            raise ValueError("acc and jerk must be (3, n_active)")
        _check(lib().nbody_correct(self._ctx, act.data_ptr(), aoff.data_ptr(), na, acc.data_ptr(), jerk.data_ptr()),
               "nbody_correct")
        self._keep = (act, aoff, acc, jerk)

    def step(self, n_block_steps: int, t_end: float) -> None:
        _check(lib().nbody_step(self._ctx, int(n_block_steps), float(t_end)), "nbody_step")

    def sync(self) -> None:
        _check(lib().nbody_sync(self._ctx), "nbody_sync")

    def status(self) -> int:
        return lib().nbody_sync(self._ctx)

    def energy(self) -> np.ndarray:
        e = np.zeros(self.nc)
        _check(lib().nbody_energy(self._ctx, e.ctypes.data), "nbody_energy")
        return e

    def diagnostics(self) -> dict:
        """Per cluster: kinetic, potential and total energy, momentum (nc, 3),
        angular momentum (nc, 3)."""
        d = np.zeros((self.nc, 8))
        _check(lib().nbody_diagnostics(self._ctx, d.ctypes.data), "nbody_diagnostics")
        return {"KE": d[:, 0].copy(), "PE": d[:, 1].copy(), "E": d[:, 0] + d[:, 1], "P": d[:, 2:5].copy(),
                "L": d[:, 5:8].copy()}

    def progress(self):
        t = np.zeros(self.nc)
        s = np.zeros(self.nc, dtype=np.int64)
        it = np.zeros(self.nc)
        _check(lib().nbody_progress(self._ctx, t.ctypes.data, s.ctypes.data, it.ctypes.data), "nbody_progress")
        return t, s, it

    def run(self, t_end: float, chunk: int = 64, max_steps: int = 1 << 40) -> int:
        """Block steps until every cluster reaches t_end (a multiple of dt_max)."""
        done = 0
        while done < max_steps:
            self.step(chunk, t_end)
            done += chunk
            t, _, _ = self.progress()
            st = self.status()
            if st != 0:
                raise NBodyError(st, "nbody_step")
            if np.all(t >= t_end):
                break
        return done

    def get_state(self) -> bytes:
        nb = ctypes.c_size_t(0)
        _check(lib().nbody_state_bytes(self._ctx, ctypes.byref(nb)), "nbody_state_bytes")
        buf = ctypes.create_string_buffer(nb.value)
        _check(lib().nbody_get_state(self._ctx, buf, nb.value), "nbody_get_state")
        return buf.raw

    def set_state(self, blob: bytes) -> None:
        buf = ctypes.create_string_buffer(blob, len(blob))
        _check(lib().nbody_set_state(self._ctx, buf, len(blob)), "nbody_set_state")

    def host_state(self) -> dict:
        """The FP64 state copied to host numpy arrays."""
        self._torch.cuda.synchronize(self.device)
        return {k: getattr(self, k).cpu().numpy().copy() for k in ("m", "x", "v", "a", "k", "t", "dt")}

    def close(self) -> None:
        if self._ctx:
            lib().nbody_destroy(self._ctx)
            self._ctx = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
