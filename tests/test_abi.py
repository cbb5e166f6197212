"""The C-ABI library loads and exports every symbol include/argus.h declares;
argument validation on the host rejects bad datasets before any GPU work.
CPU only: no compute call reaches a device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2510_11077_amd", "libargus.so")
HDR = os.path.join(ROOT, "include", "argus.h")


def declared():
    txt = open(HDR).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(argus_[a-z0-9_]+)\s*\(", txt)))


def lib():
    if not os.path.exists(LIB):
        pytest.skip("libargus.so not built")
    return C.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared()
    for n in ("argus_dataset_create", "argus_dataset_destroy", "argus_loglike",
              "argus_loglike_grad", "argus_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    L = lib()
    missing = [n for n in declared() if not hasattr(L, n)]
    assert not missing, missing


class Desc(C.Structure):
    _fields_ = [("model", C.c_int32), ("n_psr", C.c_int32), ("toa_off", C.c_void_p),
                ("t", C.c_void_p), ("y", C.c_void_p), ("sigma", C.c_void_p),
                ("pos", C.c_void_p), ("fixed", C.c_void_p), ("free_mask", C.c_void_p),
                ("t_span", C.c_double), ("s_r", C.c_double), ("s_f", C.c_double),
                ("sigma_s", C.c_double), ("freq", C.c_void_p)]


def test_descriptor_layout_matches_the_header():
    """The struct above mirrors argus_dataset_desc field by field."""
    txt = open(HDR).read()
    body = re.search(r"typedef struct \{(.*?)\} argus_dataset_desc;", txt, re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    # each declaration's names are the identifiers followed by "," or its end
    names = [n for decl in body.split(";") for n in re.findall(r"(\w+)\s*(?:,|$)", decl.strip())]
    assert names == [f for f, _ in Desc._fields_], names


def make(model=2, P=2, t=None, y=None, sig=None, pos=None, off=None, fixed=None, freq=None):
    off = np.array([0, 3, 5] if off is None else off, np.int64)
    t = np.array([1.0, 2.0, 3.0, 1.5, 2.5] if t is None else t)
    y = np.zeros_like(t) if y is None else np.asarray(y, float)
    sig = np.full_like(t, 1e-7) if sig is None else np.asarray(sig, float)
    freq = None if freq is None else np.asarray(freq, float)
    keep = [off, t, y, sig, pos, fixed, freq]
    d = Desc(model, P, off.ctypes.data, t.ctypes.data, y.ctypes.data, sig.ctypes.data,
             None if pos is None else pos.ctypes.data,
             None if fixed is None else fixed.ctypes.data, None, 3e8, 1e-6, 1e-14, 1e-20,
             None if freq is None else freq.ctypes.data)
    return d, keep


@pytest.mark.parametrize("case,code", [
    (dict(t=[1.0, 3.0, 2.0, 1.5, 2.5]), 1),          # not ascending within pulsar 0
    (dict(t=[-1.0, 2.0, 3.0, 1.5, 2.5]), 1),         # before the epoch
    (dict(sig=[1e-7, 0.0, 1e-7, 1e-7, 1e-7]), 1),    # sigma must be > 0
    (dict(y=[0, np.nan, 0, 0, 0]), 1),               # y finite
    (dict(off=[1, 3, 5]), 1),                        # off[0] must be 0
    (dict(off=[0, 4, 3]), 1),                        # decreasing offsets
    (dict(model=3), 1),                              # joint model needs positions
    (dict(model=1), 1),                              # spin model takes one pulsar
    (dict(model=7), 1),                              # unknown model
    (dict(model=4), 1),                              # DM model needs radio frequencies
    (dict(model=4, freq=[1400, 820, 0.0, 430, 2300]), 1),     # frequency must be > 0
    (dict(model=4, freq=[1400, 820, -5.0, 430, 2300]), 1),    # negative frequency
    (dict(model=4, freq=[1400, np.nan, 820, 430, 2300]), 1),  # frequency must be finite
    (dict(model=4, freq=[1400, np.inf, 820, 430, 2300]), 1),
])
def test_dataset_validation(case, code):
    L = lib()
    L.argus_last_error.restype = C.c_char_p
    d, keep = make(**case)
    h = C.c_void_p()
    rc = L.argus_dataset_create(C.byref(d), C.byref(h))
    assert rc == code, L.argus_last_error()
    assert h.value is None
    assert len(L.argus_last_error()) > 0


def test_joint_model_size_limit():
    L = lib()
    P = 64  # one more than the sequential joint kernel holds
    off = np.arange(P + 1, dtype=np.int64)
    t = np.ones(P)
    pos = np.tile([0, 0, 1.0], (P, 1))
    d, keep = make(model=3, P=P, off=off, t=t, pos=pos)
    h = C.c_void_p()
    assert L.argus_dataset_create(C.byref(d), C.byref(h)) == 4  # ARGUS_E_UNSUPPORTED


def test_null_arguments_rejected():
    L = lib()
    assert L.argus_dataset_create(None, None) == 1
    for n in ("argus_loglike", "argus_loglike_plain", "argus_loglike_terms"):
        f = getattr(L, n)
        f.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p]
        assert f(None, None, 4, None, None, None) == 1
