"""CPU oracle for the state-space PTA likelihood (FP64).

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the product path. It shares no
code with the GPU library.

* ``liboracle.so`` (argus_oracle.cpp): the Kalman recursion written out
  densely in Joseph form, templated for complex-step gradients, and the
  Rauch-Tung-Striebel smoother on its filtered and predicted moments.
* ``dense``: the same likelihood by its plain definition, log N(y; 0, C) with
  C built from closed-form covariance functions, used to pin the recursion.
* ``mlp``: FP64 NumPy surrogate network with BF16 rounding emulation + Adam.
* ``da``: delayed-acceptance Metropolis-Hastings reference.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "argus_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = False) -> str:
    """Compile liboracle.so with g++ (-O2, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
                        "-o", tmp, _SRC, "-lpthread"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _DS(C.Structure):
    _fields_ = [("model", C.c_int32), ("n_psr", C.c_int32),
                ("off", C.c_void_p), ("t", C.c_void_p), ("y", C.c_void_p),
                ("sigma", C.c_void_p), ("pos", C.c_void_p),
                ("t_span", C.c_double), ("s_r", C.c_double), ("s_f", C.c_double),
                ("sigma_s", C.c_double), ("freq", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        P = C.c_void_p
        _lib.oracle_loglike.argtypes = [P, P, C.c_int64, P, P, P, C.c_int]
        _lib.oracle_grad_cs.argtypes = [P, P, C.c_int64, P, C.c_int, C.c_double, P, C.c_int]
        _lib.oracle_trace.argtypes = [P, P, C.c_int, P, P, P, P, P, P, P]
        _lib.oracle_merged.argtypes = [P, P, P]
        _lib.oracle_model_mats.argtypes = [P, P, C.c_int, C.c_double, P, P, P]
        _lib.oracle_model_mats.restype = C.c_int
        _lib.oracle_hd.argtypes = [P, C.c_int, P]
        _lib.oracle_common_variance.argtypes = [C.c_double, C.c_double, C.c_double]
        _lib.oracle_common_variance.restype = C.c_double
        _lib.oracle_smooth_stream.argtypes = [P, P, C.c_int, P, P, P, P]
        _lib.oracle_smooth.argtypes = [P, P, C.c_int64, P, P, P, C.c_int]
        _lib.oracle_scan_filter.argtypes = [P, P, C.c_int, C.c_int, C.c_int, P, P, P]
        _lib.oracle_n_canon.argtypes = [P]
        _lib.oracle_n_canon.restype = C.c_int
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


class Dataset:
    """Holds contiguous copies of a dataset's arrays and the C descriptor."""

    def __init__(self, d):
        self.d = d
        self.model = int(d.model)
        self.n_psr = int(d.n_psr)
        self.off = np.ascontiguousarray(d.off, np.int64)
        self.t = np.ascontiguousarray(d.t, np.float64)
        self.y = np.ascontiguousarray(d.y, np.float64)
        self.sigma = np.ascontiguousarray(d.sigma, np.float64)
        self.pos = None if d.pos is None else np.ascontiguousarray(d.pos, np.float64)
        fr = getattr(d, "freq", None)
        self.freq = None if fr is None else np.ascontiguousarray(fr, np.float64)
        self.desc = _DS(self.model, self.n_psr, _ptr(self.off), _ptr(self.t), _ptr(self.y),
                        _ptr(self.sigma), _ptr(self.pos), float(d.t_span), float(d.s_r),
                        float(d.s_f), float(d.sigma_s), _ptr(self.freq))
        self.C = lib().oracle_n_canon(C.byref(self.desc))

    @property
    def n(self) -> int:
        return {1: 2, 2: 4, 4: 5}.get(self.model, 4 * self.n_psr)


def _as_ds(d) -> Dataset:
    return d if isinstance(d, Dataset) else Dataset(d)


def host_cpus() -> dict:
    """The host's CPUs as this process sees them: nproc (os.cpu_count), the
    CPUs it may run on (affinity), the cgroup CPU quota if one is set, the
    CPU model name, and 'usable' = the smaller of affinity and quota."""
    nproc = os.cpu_count() or 1
    try:
        aff = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        aff = nproc
    quota = None
    try:
        with open("/sys/fs/cgroup/cpu.max") as fh:
            q, period = fh.read().split()[:2]
        if q != "max":
            quota = int(q) / int(period)
    except (OSError, ValueError):
        pass
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    usable = aff if quota is None else min(aff, max(1, int(quota)))
    return {"nproc": nproc, "affinity": aff, "cgroup_quota": quota, "model": model,
            "usable": max(1, usable)}


def default_threads() -> int:
    """One thread per CPU this process can use (affinity and cgroup quota)."""
    return host_cpus()["usable"]


def loglike(d, canon, nthreads=None, per_psr=False):
    """log L for canonical parameter rows canon [S, C] -> (logl [S], status [S]
    [, per-pulsar terms [S, P]])."""
    ds = _as_ds(d)
    c = np.ascontiguousarray(np.atleast_2d(canon), np.float64)
    assert c.shape[1] == ds.C
    S = c.shape[0]
    out = np.empty(S)
    st = np.empty(S, np.int32)
    pp = np.empty((S, ds.n_psr)) if per_psr else None
    lib().oracle_loglike(C.byref(ds.desc), _ptr(c), S, _ptr(out), _ptr(st), _ptr(pp),
                         nthreads or default_threads())
    return (out, st, pp) if per_psr else (out, st)


def grad_cs(d, canon, which=None, h=1e-30, nthreads=None):
    """Complex-step d logL / d canon[:, which] -> [S, len(which)]."""
    ds = _as_ds(d)
    c = np.ascontiguousarray(np.atleast_2d(canon), np.float64)
    which = np.arange(ds.C, dtype=np.int32) if which is None else np.ascontiguousarray(which, np.int32)
    S = c.shape[0]
    g = np.empty((S, which.size))
    lib().oracle_grad_cs(C.byref(ds.desc), _ptr(c), S, _ptr(which), which.size, h, _ptr(g),
                         nthreads or default_threads())
    return g


def trace(d, canon, q=0):
    """Per-step record of one filter: dict with e, S, x, Pf, Pp, ll, status."""
    ds = _as_ds(d)
    c = np.ascontiguousarray(canon, np.float64).ravel()
    N = int(ds.off[-1]) if ds.model == 3 else int(ds.off[q + 1] - ds.off[q])
    n = ds.n
    r = dict(e=np.empty(N), S=np.empty(N), x=np.empty((N, n)), Pf=np.empty((N, n, n)),
             Pp=np.empty((N, n, n)))
    ll = np.empty(1)
    st = np.empty(1, np.int32)
    lib().oracle_trace(C.byref(ds.desc), _ptr(c), q, _ptr(r["e"]), _ptr(r["S"]), _ptr(r["x"]),
                       _ptr(r["Pf"]), _ptr(r["Pp"]), _ptr(ll), _ptr(st))
    r["ll"], r["status"] = float(ll[0]), int(st[0])
    return r


def smooth(d, canon, nthreads=None):
    """Rauch-Tung-Striebel smoothed moments of each TOA's own pulsar state
    -> (mean [S, N, nc], var [S, N, nc], status [S]); nc = 2 (model 1) or 4
    ([r, f, a, g]); NaN where that pulsar's filter failed."""
    ds = _as_ds(d)
    c = np.ascontiguousarray(np.atleast_2d(canon), np.float64)
    assert c.shape[1] == ds.C
    S, N = c.shape[0], int(ds.off[-1])
    nc = {1: 2, 4: 5}.get(ds.model, 4)
    mean = np.empty((S, N, nc))
    var = np.empty((S, N, nc))
    st = np.empty(S, np.int32)
    lib().oracle_smooth(C.byref(ds.desc), _ptr(c), S, _ptr(mean), _ptr(var), _ptr(st),
                        nthreads or default_threads())
    return mean, var, st


def smooth_stream(d, canon, q=0):
    """Smoothed mean xs [N, n] and covariance Ps [N, n, n] of one filter's
    full state, in stream order (pulsar q, or the joint merged stream)."""
    ds = _as_ds(d)
    c = np.ascontiguousarray(canon, np.float64).ravel()
    N = int(ds.off[-1]) if ds.model == 3 else int(ds.off[q + 1] - ds.off[q])
    n = ds.n
    xs, Ps = np.empty((N, n)), np.empty((N, n, n))
    ll = np.empty(1)
    st = np.empty(1, np.int32)
    lib().oracle_smooth_stream(C.byref(ds.desc), _ptr(c), q, _ptr(xs), _ptr(Ps), _ptr(ll),
                               _ptr(st))
    return dict(xs=xs, Ps=Ps, ll=float(ll[0]), status=int(st[0]))


def scan_filter(d, canon, q=0, order=0, nchunk=1):
    """Filtered moments of pulsar q by the associative scan (per-pulsar
    models) in evaluation order 0 (left fold), 1 (recursive doubling) or 2
    (nchunk chunks) -> dict xs [N, n], Ps [N, n, n], ll."""
    ds = _as_ds(d)
    assert ds.model != 3
    c = np.ascontiguousarray(canon, np.float64).ravel()
    N = int(ds.off[q + 1] - ds.off[q])
    n = ds.n
    xs, Ps = np.empty((N, n)), np.empty((N, n, n))
    ll = np.empty(1)
    lib().oracle_scan_filter(C.byref(ds.desc), _ptr(c), q, order, nchunk, _ptr(xs), _ptr(Ps),
                             _ptr(ll))
    return dict(xs=xs, Ps=Ps, ll=float(ll[0]))


def merged_order(d):
    ds = _as_ds(d)
    N = int(ds.off[-1])
    idx = np.empty(N, np.int64)
    psr = np.empty(N, np.int32)
    lib().oracle_merged(C.byref(ds.desc), _ptr(idx), _ptr(psr))
    return idx, psr


def model_mats(d, canon, q, dt):
    """(F(dt), Q(dt), P0) of the filter for pulsar q (or the joint model)."""
    ds = _as_ds(d)
    c = np.ascontiguousarray(canon, np.float64).ravel()
    n = ds.n
    F, Q, P0 = np.empty((n, n)), np.empty((n, n)), np.empty((n, n))
    lib().oracle_model_mats(C.byref(ds.desc), _ptr(c), q, float(dt), _ptr(F), _ptr(Q), _ptr(P0))
    return F, Q, P0


def hd(pos):
    pos = np.ascontiguousarray(pos, np.float64)
    P = pos.shape[0]
    G = np.empty((P, P))
    lib().oracle_hd(_ptr(pos), P, _ptr(G))
    return G


def common_variance(log10A, gamma, t_span):
    return lib().oracle_common_variance(float(log10A), float(gamma), float(t_span))
