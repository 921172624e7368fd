"""Python binding of the SRM C-ABI library (libsrm.so): argument marshalling only.

Every step of the EM sweep runs in the library's HIP kernels; this module
allocates the caller-owned device workspace with PyTorch, passes pointers, and
converts results.  Importing it raises ImportError when libsrm.so has not been
built: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
import time
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsrm.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "srm.h")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python -m paper_1608_04647_amd.build`")

# PyTorch ships its own HIP runtime.  Loading it first makes libsrm.so bind to
# that same runtime (by soname); loaded the other way round, the process would
# hold two HIP runtimes and the library's streams would not see torch's device
# state.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

SRM_OK, SRM_E_ARG, SRM_E_WORKSPACE, SRM_E_HIP, SRM_E_RANK, SRM_E_NOTPD, \
    SRM_E_NONFINITE, SRM_E_STATE = range(8)
STATUS_NAMES = {0: "SRM_OK", 1: "SRM_E_ARG", 2: "SRM_E_WORKSPACE", 3: "SRM_E_HIP",
                4: "SRM_E_RANK", 5: "SRM_E_NOTPD", 6: "SRM_E_NONFINITE", 7: "SRM_E_STATE"}
PREC = {"fp32": 0, "bf16": 1, "bf16x2": 2}
SRM_NO_GRAPH, SRM_NO_W0_CHECK, SRM_TWO_PASS, SRM_X_HOST, SRM_ZSCORE, SRM_GRAM, \
    SRM_AUTOTUNE = 1, 2, 4, 8, 16, 32, 64
KERNELS = {0: "ring", 1: "staged"}


SWEEPS = {0: "one_pass", 1: "two_pass", 2: "gram"}


class SrmDesc(ctypes.Structure):
    _fields_ = [("n_subjects", ctypes.c_int32), ("v", ctypes.POINTER(ctypes.c_int64)),
                ("t", ctypes.c_int64), ("k", ctypes.c_int32), ("prec", ctypes.c_int),
                ("flags", ctypes.c_uint32), ("hip_stream", ctypes.c_void_p)]


class SrmInfo(ctypes.Structure):
    _fields_ = [("sweep", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("k_padded", ctypes.c_int32), ("n_ranges", ctypes.c_int32),
                ("n_slices", ctypes.c_int32), ("reserved", ctypes.c_int32 * 3),
                ("ldt", ctypes.c_int64), ("workspace_bytes", ctypes.c_size_t)]


class SrmTuning(ctypes.Structure):
    _fields_ = [("sweep_kernel", ctypes.c_int32), ("sweep_wgs", ctypes.c_int32),
                ("chunk_rows", ctypes.c_int32), ("reduce_wgs", ctypes.c_int32),
                ("mphase_rounds", ctypes.c_int32), ("reserved", ctypes.c_int32 * 3)]

    FIELDS = ("sweep_kernel", "sweep_wgs", "chunk_rows", "reduce_wgs", "mphase_rounds")

    def as_dict(self) -> dict:
        return {f: int(getattr(self, f)) for f in self.FIELDS}

    @classmethod
    def from_dict(cls, d: dict) -> "SrmTuning":
        t = cls()
        for f in cls.FIELDS:
            setattr(t, f, int(d[f]))
        return t


_P = ctypes.c_void_p
_I32, _I64, _SZ, _U64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_uint64
_DP = ctypes.POINTER(ctypes.c_double)
_sigs = {
    "srm_workspace_size": (ctypes.c_int, [ctypes.POINTER(SrmDesc), ctypes.POINTER(_SZ)]),
    "srm_init": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.POINTER(SrmDesc), _P, _P, _U64, _P,
                                _SZ]),
    "srm_init_begin": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.POINTER(SrmDesc), _U64, _P,
                                      _SZ]),
    "srm_ingest": (ctypes.c_int, [_P, _I32, _P, _P]),
    "srm_init_end": (ctypes.c_int, [_P]),
    "srm_get_info": (ctypes.c_int, [_P, ctypes.POINTER(SrmInfo)]),
    "srm_em_step": (ctypes.c_int, [_P, _DP]),
    "srm_fit": (ctypes.c_int, [_P, _I32, _DP]),
    "srm_profile": (ctypes.c_int, [_P, _I32, _DP]),
    "srm_transform": (ctypes.c_int, [_P, _I32, _P, _I64, _P]),
    "srm_transform_static": (ctypes.c_int, [_P, _I32, _P, _I64, _P]),
    "srm_map": (ctypes.c_int, [_P, _I32, _I32, _P, _I64, _P]),
    "srm_get_w": (ctypes.c_int, [_P, _I32, _P]),
    "srm_get_s": (ctypes.c_int, [_P, _P]),
    "srm_get_rho2": (ctypes.c_int, [_P, _DP]),
    "srm_get_sigma_s": (ctypes.c_int, [_P, _DP]),
    "srm_get_mu": (ctypes.c_int, [_P, _I32, _P]),
    "srm_get_scale": (ctypes.c_int, [_P, _I32, _P]),
    "srm_get_state": (ctypes.c_int, [_P, _P, ctypes.POINTER(_SZ)]),
    "srm_set_state": (ctypes.c_int, [_P, _P, _SZ]),
    "srm_get_loglik": (ctypes.c_int, [_P, _DP, _I32, ctypes.POINTER(_I32)]),
    "srm_iterations": (ctypes.c_int, [_P, ctypes.POINTER(_I32)]),
    "srm_get_tuning": (ctypes.c_int, [_P, ctypes.POINTER(SrmTuning)]),
    "srm_set_tuning": (ctypes.c_int, [_P, ctypes.POINTER(SrmTuning)]),
    "srm_tuning_candidates": (ctypes.c_int, [_P, ctypes.POINTER(SrmTuning), _I32,
                                             ctypes.POINTER(_I32)]),
    "srm_autotune": (ctypes.c_int, [_P, _I32, ctypes.POINTER(SrmTuning), _DP]),
    "srm_last_error": (ctypes.c_char_p, []),
    "srm_free": (None, [_P]),
}
for _name, (_res, _args) in _sigs.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class SRMError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _check(st: int):
    if st != SRM_OK:
        raise SRMError(st, _lib.srm_last_error().decode())


def lib() -> ctypes.CDLL:
    return _lib


def make_desc(v: Sequence[int], t: int, k: int, prec: str = "fp32", flags: int = 0):
    varr = (ctypes.c_int64 * len(v))(*[int(x) for x in v])
    d = SrmDesc(len(v), ctypes.cast(varr, ctypes.POINTER(ctypes.c_int64)), int(t), int(k),
                PREC[prec] if isinstance(prec, str) else int(prec), int(flags), None)
    d._keep = varr
    return d


def workspace_size(v: Sequence[int], t: int, k: int, prec: str = "fp32") -> int:
    d = make_desc(v, t, k, prec)
    n = _SZ()
    _check(_lib.srm_workspace_size(ctypes.byref(d), ctypes.byref(n)))
    return int(n.value)


class SRM:
    """One SRM fit on the current HIP device.

    X: list of N float32 arrays (v_i x t): torch CUDA tensors are used in
    place, anything else is uploaded (or, with stream_from_host, streamed
    through the library's staging buffers one subject at a time).  W0: list of
    N float64 host arrays (v_i x k, orthonormal columns), or None: the library
    then draws each subject's random orthonormal start from `seed` (entries of
    the list may also be None).  zscore standardises each voxel after
    demeaning; gram selects the sample-space iteration on G_i = Xhat_i^T Xhat_i.

    SRM.begin(v, t, k, ...) returns a fit awaiting its subjects: ingest(i, X_i,
    W0_i) each one (any order), then end()."""

    def __init__(self, X, k: int, prec: str = "fp32", W0=None, flags: int = 0,
                 seed: int = 0, stream_from_host: bool = False, zscore: bool = False,
                 gram: bool = False, autotune: bool = False):
        torch = self._setup(flags | (SRM_AUTOTUNE if autotune else 0), stream_from_host,
                            zscore, gram)
        xs = [self._prep_x(x) for x in X]
        self._open([int(x.shape[0]) for x in xs], int(xs[0].shape[1]), k, prec)
        w0 = None if W0 is None else [None if w is None else
                                      np.ascontiguousarray(w, dtype=np.float64) for w in W0]
        xptr = (_P * self.N)(*[(x.ctypes.data if self._host else x.data_ptr()) for x in xs])
        wptr = None if w0 is None else (_P * self.N)(*[(w.ctypes.data if w is not None else None)
                                                       for w in w0])
        torch.cuda.synchronize()
        ctx = _P()
        t0 = time.perf_counter()
        _check(_lib.srm_init(ctypes.byref(ctx), ctypes.byref(self._desc), xptr, wptr,
                             int(seed), _P(self._ws.data_ptr()), self.workspace_bytes))
        # srm_init returns after its device work (it reads the device status)
        self.init_seconds = time.perf_counter() - t0
        self._ctx = ctx

    @classmethod
    def begin(cls, v, t: int, k: int, prec: str = "fp32", flags: int = 0, seed: int = 0,
              stream_from_host: bool = False, zscore: bool = False, gram: bool = False,
              autotune: bool = False):
        """A fit awaiting its subjects (srm_init_begin)."""
        self = cls.__new__(cls)
        self._setup(flags | (SRM_AUTOTUNE if autotune else 0), stream_from_host, zscore, gram)
        self._open([int(x) for x in v], int(t), k, prec)
        ctx = _P()
        self._t0 = time.perf_counter()
        _check(_lib.srm_init_begin(ctypes.byref(ctx), ctypes.byref(self._desc), int(seed),
                                   _P(self._ws.data_ptr()), self.workspace_bytes))
        self._ctx = ctx
        return self

    def ingest(self, i: int, X_i, W0_i=None):
        """Store subject i (srm_ingest); X_i and W0_i may be released afterwards."""
        x = self._prep_x(X_i)
        w = None if W0_i is None else np.ascontiguousarray(W0_i, dtype=np.float64)
        if not self._host:
            self._torch.cuda.synchronize()  # torch's upload precedes the library's stream
        _check(_lib.srm_ingest(self._ctx, int(i),
                               _P(x.ctypes.data if self._host else x.data_ptr()),
                               None if w is None else _P(w.ctypes.data)))

    def end(self):
        """srm_init_end: every subject ingested; runs the first E-step."""
        t0 = time.perf_counter()
        _check(_lib.srm_init_end(self._ctx))
        self.end_seconds = time.perf_counter() - t0
        self.init_seconds = time.perf_counter() - self._t0
        return self

    def _setup(self, flags, stream_from_host, zscore, gram):
        import torch
        if not torch.cuda.is_available():
            raise SRMError(SRM_E_HIP, "no HIP device visible")
        self._torch = torch
        self._dev = torch.device("cuda", torch.cuda.current_device())
        self._host = bool(stream_from_host)
        self._flags = int(flags) | (SRM_ZSCORE if zscore else 0) | (SRM_GRAM if gram else 0) \
            | (SRM_X_HOST if stream_from_host else 0)
        self._ctx = None
        return torch

    def _prep_x(self, x):
        torch = self._torch
        if self._host:
            return np.ascontiguousarray(x, dtype=np.float32)
        if isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float32 \
                and x.is_contiguous():
            return x
        return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float32)).to(self._dev)

    def _open(self, v, t, k, prec):
        self.N = len(v)
        self.v = list(v)
        self.t = int(t)
        self.k = int(k)
        self.prec = prec
        self._desc = make_desc(self.v, self.t, self.k, prec, self._flags)
        n = _SZ()
        _check(_lib.srm_workspace_size(ctypes.byref(self._desc), ctypes.byref(n)))
        self.workspace_bytes = int(n.value)
        self._ws = self._torch.empty(self.workspace_bytes, dtype=self._torch.uint8,
                                     device=self._dev)

    def info(self) -> dict:
        """srm_get_info: the sweep, whether the graph ran, the plan's sizes."""
        inf = SrmInfo()
        _check(_lib.srm_get_info(self._ctx, ctypes.byref(inf)))
        return {"sweep": SWEEPS.get(inf.sweep, inf.sweep), "graph": bool(inf.graph),
                "k_padded": inf.k_padded, "n_ranges": inf.n_ranges, "n_slices": inf.n_slices,
                "ldt": inf.ldt, "workspace_bytes": inf.workspace_bytes}

    # -- launch shapes -----------------------------------------------------
    def tuning(self) -> dict:
        t = SrmTuning()
        _check(_lib.srm_get_tuning(self._ctx, ctypes.byref(t)))
        return t.as_dict()

    def set_tuning(self, d: dict):
        _check(_lib.srm_set_tuning(self._ctx, ctypes.byref(SrmTuning.from_dict(d))))

    def tuning_candidates(self) -> list:
        n = _I32()
        _check(_lib.srm_tuning_candidates(self._ctx, None, 0, ctypes.byref(n)))
        arr = (SrmTuning * max(n.value, 1))()
        _check(_lib.srm_tuning_candidates(self._ctx, arr, n.value, ctypes.byref(n)))
        return [arr[i].as_dict() for i in range(n.value)]

    def autotune(self, trials: int = 2):
        """srm_autotune: times the candidates, keeps the fastest; returns
        (shape, ms per iteration)."""
        t = SrmTuning()
        ms = ctypes.c_double()
        _check(_lib.srm_autotune(self._ctx, int(trials), ctypes.byref(t), ctypes.byref(ms)))
        return t.as_dict(), ms.value

    # -- iteration ---------------------------------------------------------
    def fit(self, n_iter: int) -> np.ndarray:
        ll = np.zeros(max(n_iter, 1))
        _check(_lib.srm_fit(self._ctx, int(n_iter), ll.ctypes.data_as(_DP)))
        return ll[:n_iter]

    PHASES = ("mphase", "ephase", "polar", "ereduce", "posterior", "fused", "gram")

    def profile(self, n_iter: int) -> dict:
        """Milliseconds per kernel phase summed over n_iter iterations, from HIP
        events on the library's stream (direct launches)."""
        ms = np.zeros(len(self.PHASES))
        _check(_lib.srm_profile(self._ctx, int(n_iter), ms.ctypes.data_as(_DP)))
        return dict(zip(self.PHASES, ms.tolist()))

    def em_step(self) -> float:
        ll = ctypes.c_double()
        _check(_lib.srm_em_step(self._ctx, ctypes.byref(ll)))
        return ll.value

    # -- results -----------------------------------------------------------
    def _sync(self):
        self._torch.cuda.synchronize()

    def W(self, i: int):
        out = self._torch.empty((self.v[i], self.k), dtype=self._torch.float32, device=self._dev)
        _check(_lib.srm_get_w(self._ctx, int(i), _P(out.data_ptr())))
        self._sync()
        return out

    def S(self):
        out = self._torch.empty((self.k, self.t), dtype=self._torch.float32, device=self._dev)
        _check(_lib.srm_get_s(self._ctx, _P(out.data_ptr())))
        self._sync()
        return out

    def rho2(self) -> np.ndarray:
        out = np.zeros(self.N)
        _check(_lib.srm_get_rho2(self._ctx, out.ctypes.data_as(_DP)))
        return out

    def sigma_s(self) -> np.ndarray:
        out = np.zeros((self.k, self.k))
        _check(_lib.srm_get_sigma_s(self._ctx, out.ctypes.data_as(_DP)))
        return out

    def mu(self, i: int):
        out = self._torch.empty(self.v[i], dtype=self._torch.float64, device=self._dev)
        _check(_lib.srm_get_mu(self._ctx, int(i), _P(out.data_ptr())))
        self._sync()
        return out

    def scale(self, i: int):
        out = self._torch.empty(self.v[i], dtype=self._torch.float64, device=self._dev)
        _check(_lib.srm_get_scale(self._ctx, int(i), _P(out.data_ptr())))
        self._sync()
        return out

    def get_state(self) -> bytes:
        """Checkpoint of everything an iteration carries to the next."""
        n = _SZ()
        _check(_lib.srm_get_state(self._ctx, None, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        _check(_lib.srm_get_state(self._ctx, ctypes.cast(buf, _P), ctypes.byref(n)))
        return buf.raw[:n.value]

    def set_state(self, blob: bytes):
        buf = ctypes.create_string_buffer(bytes(blob), len(blob))
        _check(_lib.srm_set_state(self._ctx, ctypes.cast(buf, _P), len(blob)))

    def loglik(self) -> np.ndarray:
        cnt = _I32()
        _check(_lib.srm_get_loglik(self._ctx, None, 0, ctypes.byref(cnt)))
        out = np.zeros(max(cnt.value, 1))
        _check(_lib.srm_get_loglik(self._ctx, out.ctypes.data_as(_DP), cnt.value,
                                   ctypes.byref(cnt)))
        return out[:cnt.value]

    def iterations(self) -> int:
        n = _I32()
        _check(_lib.srm_iterations(self._ctx, ctypes.byref(n)))
        return n.value

    def transform(self, i: int, X_new):
        torch = self._torch
        x = X_new if (isinstance(X_new, torch.Tensor) and X_new.is_cuda) else \
            torch.as_tensor(np.ascontiguousarray(X_new, dtype=np.float32)).to(self._dev)
        x = x.to(torch.float32).contiguous()
        out = torch.empty((self.k, x.shape[1]), dtype=torch.float32, device=self._dev)
        self._sync()
        _check(_lib.srm_transform(self._ctx, int(i), _P(x.data_ptr()), int(x.shape[1]),
                                  _P(out.data_ptr())))
        self._sync()
        return out

    def transform_static(self, i: int, X_new, out=None):
        """srm_transform_static: as transform, its partials in the library's
        static device scratch (no allocation in the call); out, if given, is a
        k x t_new float32 device tensor."""
        torch = self._torch
        x = X_new if (isinstance(X_new, torch.Tensor) and X_new.is_cuda) else \
            torch.as_tensor(np.ascontiguousarray(X_new, dtype=np.float32)).to(self._dev)
        x = x.to(torch.float32).contiguous()
        if out is None:
            out = torch.empty((self.k, x.shape[1]), dtype=torch.float32, device=self._dev)
        self._sync()
        _check(_lib.srm_transform_static(self._ctx, int(i), _P(x.data_ptr()), int(x.shape[1]),
                                         _P(out.data_ptr())))
        self._sync()
        return out

    def map(self, i: int, j: int, X_new):
        """Subject i's samples mapped into subject j's (demeaned) voxel space:
        W_j W_i^T (X_new - mu_i 1^T)."""
        torch = self._torch
        x = X_new if (isinstance(X_new, torch.Tensor) and X_new.is_cuda) else \
            torch.as_tensor(np.ascontiguousarray(X_new, dtype=np.float32)).to(self._dev)
        x = x.to(torch.float32).contiguous()
        out = torch.empty((self.v[j], x.shape[1]), dtype=torch.float32, device=self._dev)
        self._sync()
        _check(_lib.srm_map(self._ctx, int(i), int(j), _P(x.data_ptr()), int(x.shape[1]),
                            _P(out.data_ptr())))
        self._sync()
        return out

    def close(self):
        if getattr(self, "_ctx", None):
            _lib.srm_free(self._ctx)
            self._ctx = None
            self._torch.cuda.synchronize()
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
