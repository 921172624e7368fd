"""C-ABI checks that need no GPU: the library loads, exports every entry point
include/srm.h declares, and rejects invalid arguments before touching HIP."""
import ctypes
import os
import re

import numpy as np
import pytest

srm = pytest.importorskip("paper_1608_04647_amd.srm")


def _declared():
    txt = open(srm.HEADER_PATH).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(srm_[a-z_0-9]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported():
    names = _declared()
    assert "srm_init" in names and "srm_fit" in names and "srm_transform" in names
    for n in names:
        assert hasattr(srm.lib(), n), n


def _desc(v=(100, 120), t=50, k=5, prec="fp32"):
    return srm.make_desc(v, t, k, prec)


def _ws(d):
    n = ctypes.c_size_t()
    st = srm.lib().srm_workspace_size(ctypes.byref(d), ctypes.byref(n))
    return st, n.value


def test_workspace_size_valid_and_monotone():
    st, a = _ws(_desc())
    assert st == srm.SRM_OK and a > 0
    _, b = _ws(_desc(v=(100, 120, 300)))
    _, c = _ws(_desc(prec="bf16x2"))
    _, d = _ws(_desc(prec="bf16"))
    assert b > a and c > d
    # the stored data alone: padded rows x padded TRs x bytes per element
    assert a >= (128 + 128) * 64 * 4


@pytest.mark.parametrize("kw,code", [
    (dict(k=0), srm.SRM_E_ARG),
    (dict(k=129), srm.SRM_E_ARG),
    (dict(t=1), srm.SRM_E_ARG),
    (dict(k=60, t=50), srm.SRM_E_ARG),        # k > t
    (dict(v=(100, 3), k=5), srm.SRM_E_ARG),   # k > v_i
    (dict(prec=7), srm.SRM_E_ARG),
])
def test_invalid_descriptors(kw, code):
    st, _ = _ws(_desc(**kw))
    assert st == code
    assert srm.lib().srm_last_error().decode() != ""


def test_zero_subjects_and_null_pointers():
    d = _desc()
    d.n_subjects = 0
    assert _ws(d)[0] == srm.SRM_E_ARG
    n = ctypes.c_size_t()
    assert srm.lib().srm_workspace_size(None, ctypes.byref(n)) == srm.SRM_E_ARG
    d = _desc()
    assert srm.lib().srm_workspace_size(ctypes.byref(d), None) == srm.SRM_E_ARG


def _init(d, X, W0, ws, nbytes):
    ctx = ctypes.c_void_p()
    return srm.lib().srm_init(ctypes.byref(ctx), ctypes.byref(d), X, W0, 0, ws, nbytes), ctx


def test_init_argument_errors_before_any_device_call():
    d = _desc()
    _, nbytes = _ws(d)
    fake = (ctypes.c_void_p * 2)(0x1000, 0x2000)  # never dereferenced
    w = [np.linalg.qr(np.random.default_rng(i).standard_normal((v, 5)))[0]
         for i, v in enumerate((100, 120))]
    wp = (ctypes.c_void_p * 2)(*[x.ctypes.data for x in w])
    assert _init(d, None, wp, ctypes.c_void_p(0x10000), nbytes)[0] == srm.SRM_E_ARG
    nullx = (ctypes.c_void_p * 2)(0x1000, 0)
    assert _init(d, nullx, wp, ctypes.c_void_p(0x10000), nbytes)[0] == srm.SRM_E_ARG
    assert _init(d, fake, wp, None, nbytes)[0] == srm.SRM_E_WORKSPACE
    assert _init(d, fake, wp, ctypes.c_void_p(0x10001), nbytes)[0] == srm.SRM_E_WORKSPACE
    assert _init(d, fake, wp, ctypes.c_void_p(0x10000), nbytes - 1)[0] == srm.SRM_E_WORKSPACE
    # W0 with non-orthonormal columns
    bad = [x * 1.001 for x in w]
    bp = (ctypes.c_void_p * 2)(*[x.ctypes.data for x in bad])
    st, _ = _init(d, fake, bp, ctypes.c_void_p(0x10000), nbytes)
    assert st == srm.SRM_E_ARG
    assert "orthonormal" in srm.lib().srm_last_error().decode()


def test_incremental_init_argument_errors_before_any_device_call():
    lib = srm.lib()
    d = _desc()
    _, nbytes = _ws(d)
    ctx = ctypes.c_void_p()
    assert lib.srm_init_begin(None, ctypes.byref(d), 0, ctypes.c_void_p(0x10000),
                              nbytes) == srm.SRM_E_ARG
    assert lib.srm_init_begin(ctypes.byref(ctx), None, 0, ctypes.c_void_p(0x10000),
                              nbytes) == srm.SRM_E_ARG
    assert lib.srm_init_begin(ctypes.byref(ctx), ctypes.byref(d), 0, None,
                              nbytes) == srm.SRM_E_WORKSPACE
    assert lib.srm_init_begin(ctypes.byref(ctx), ctypes.byref(d), 0,
                              ctypes.c_void_p(0x10000), nbytes - 1) == srm.SRM_E_WORKSPACE
    bad = _desc(k=0)
    assert lib.srm_init_begin(ctypes.byref(ctx), ctypes.byref(bad), 0,
                              ctypes.c_void_p(0x10000), nbytes) == srm.SRM_E_ARG
    assert not ctx.value
    assert lib.srm_ingest(None, 0, None, None) == srm.SRM_E_ARG
    assert lib.srm_init_end(None) == srm.SRM_E_ARG
    info = srm.SrmInfo()
    assert lib.srm_get_info(None, ctypes.byref(info)) == srm.SRM_E_ARG


def test_calls_on_null_context():
    lib = srm.lib()
    assert lib.srm_fit(None, 1, None) == srm.SRM_E_ARG
    assert lib.srm_em_step(None, None) == srm.SRM_E_ARG
    assert lib.srm_get_w(None, 0, None) == srm.SRM_E_ARG
    assert lib.srm_transform(None, 0, None, 1, None) == srm.SRM_E_ARG
    assert lib.srm_map(None, 0, 1, None, 1, None) == srm.SRM_E_ARG
    assert lib.srm_get_scale(None, 0, None) == srm.SRM_E_ARG
    n = ctypes.c_size_t(0)
    assert lib.srm_get_state(None, None, ctypes.byref(n)) == srm.SRM_E_ARG
    assert lib.srm_set_state(None, None, 0) == srm.SRM_E_ARG
    assert lib.srm_transform_static(None, 0, None, 1, None) == srm.SRM_E_ARG
    t = srm.SrmTuning()
    cnt = ctypes.c_int32()
    assert lib.srm_get_tuning(None, ctypes.byref(t)) == srm.SRM_E_ARG
    assert lib.srm_set_tuning(None, ctypes.byref(t)) == srm.SRM_E_ARG
    assert lib.srm_tuning_candidates(None, None, 0, ctypes.byref(cnt)) == srm.SRM_E_ARG
    assert lib.srm_autotune(None, 2, None, None) == srm.SRM_E_ARG
    lib.srm_free(None)


def test_binding_refuses_missing_device():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    with pytest.raises(srm.SRMError):
        srm.SRM([np.zeros((10, 8), np.float32)], 2)


def test_single_hip_runtime_in_process():
    """The binding loads PyTorch's HIP runtime before libsrm.so, so the
    process maps exactly one libamdhip64 (two runtimes would not share
    streams or device state)."""
    maps = [l.split()[-1] for l in open("/proc/self/maps") if "libamdhip64" in l]
    assert len(set(maps)) == 1, sorted(set(maps))
