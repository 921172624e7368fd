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
SRM_NO_GRAPH, SRM_NO_W0_CHECK, SRM_TWO_PASS, SRM_X_HOST, SRM_ZSCORE, SRM_GRAM = \
    1, 2, 4, 8, 16, 32


class SrmDesc(ctypes.Structure):
    _fields_ = [("n_subjects", ctypes.c_int32), ("v", ctypes.POINTER(ctypes.c_int64)),
                ("t", ctypes.c_int64), ("k", ctypes.c_int32), ("prec", ctypes.c_int),
                ("flags", ctypes.c_uint32), ("hip_stream", ctypes.c_void_p)]


_P = ctypes.c_void_p
_I32, _I64, _SZ = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
_DP = ctypes.POINTER(ctypes.c_double)
_sigs = {
    "srm_workspace_size": (ctypes.c_int, [ctypes.POINTER(SrmDesc), ctypes.POINTER(_SZ)]),
    "srm_init": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.POINTER(SrmDesc), _P, _P, _P, _SZ]),
    "srm_em_step": (ctypes.c_int, [_P, _DP]),
    "srm_fit": (ctypes.c_int, [_P, _I32, _DP]),
    "srm_profile": (ctypes.c_int, [_P, _I32, _DP]),
    "srm_transform": (ctypes.c_int, [_P, _I32, _P, _I64, _P]),
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


def random_init(v: Sequence[int], k: int, seed: int = 0) -> List[np.ndarray]:
    """Random orthonormal starting maps (Algorithm 1 initialisation): Q of the
    QR of a seeded Gaussian, one per subject."""
    out = []
    for i, vi in enumerate(v):
        g = np.random.default_rng([seed, i]).standard_normal((int(vi), k))
        q, r = np.linalg.qr(g)
        out.append(q * np.where(np.diag(r) < 0, -1.0, 1.0))
    return out


class SRM:
    """One SRM fit on the current HIP device.

    X: list of N float32 arrays (v_i x t): torch CUDA tensors are used in
    place, anything else is uploaded (or, with stream_from_host, streamed
    through the library's staging area one subject at a time).  W0: list of
    N float64 host arrays (v_i x k, orthonormal columns); None draws random
    orthonormal maps.  zscore standardises each voxel after demeaning; gram
    selects the sample-space iteration on G_i = Xhat_i^T Xhat_i."""

    def __init__(self, X, k: int, prec: str = "fp32", W0=None, flags: int = 0,
                 seed: int = 0, stream_from_host: bool = False, zscore: bool = False,
                 gram: bool = False):
        import torch
        if not torch.cuda.is_available():
            raise SRMError(SRM_E_HIP, "no HIP device visible")
        self._torch = torch
        dev = torch.device("cuda", torch.cuda.current_device())
        xs = []
        if zscore:
            flags |= SRM_ZSCORE
        if gram:
            flags |= SRM_GRAM
        if stream_from_host:
            flags |= SRM_X_HOST
            for x in X:
                xs.append(np.ascontiguousarray(x, dtype=np.float32))
        else:
            for x in X:
                if isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float32 \
                        and x.is_contiguous():
                    xs.append(x)
                else:
                    xs.append(torch.as_tensor(np.ascontiguousarray(x, dtype=np.float32)).to(dev))
        self.N = len(xs)
        self.v = [int(x.shape[0]) for x in xs]
        self.t = int(xs[0].shape[1])
        self.k = int(k)
        self.prec = prec
        if W0 is None:
            W0 = random_init(self.v, self.k, seed)
        w0 = [np.ascontiguousarray(w, dtype=np.float64) for w in W0]
        self._desc = make_desc(self.v, self.t, self.k, prec, flags)
        n = _SZ()
        _check(_lib.srm_workspace_size(ctypes.byref(self._desc), ctypes.byref(n)))
        self.workspace_bytes = int(n.value)
        self._ws = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=dev)
        xptr = (_P * self.N)(*[(x.ctypes.data if stream_from_host else x.data_ptr())
                               for x in xs])
        wptr = (_P * self.N)(*[w.ctypes.data for w in w0])
        torch.cuda.synchronize()
        ctx = _P()
        t0 = time.perf_counter()
        _check(_lib.srm_init(ctypes.byref(ctx), ctypes.byref(self._desc), xptr, wptr,
                             _P(self._ws.data_ptr()), self.workspace_bytes))
        # srm_init returns after its device work (it reads the device status)
        self.init_seconds = time.perf_counter() - t0
        self._ctx = ctx
        self._dev = dev

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
