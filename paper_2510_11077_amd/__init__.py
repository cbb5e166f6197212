"""Python binding of libargus (include/argus.h): argument marshalling only.

Every step of the likelihood, its gradient and the surrogate runs in the HIP
kernels of libargus.so; PyTorch supplies device memory and streams. The
library must be built in-tree (``python paper_2510_11077_amd/build.py``);
importing this package fails loudly when it is missing.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libargus.so")

M1_SPIN, M2_PSR4, M3_JOINT_HD, M4_PSR5_DM = 1, 2, 3, 4
S_NONPD, S_NONFINITE = 1, 2

if not os.path.exists(LIB_PATH):
    raise ImportError("libargus.so is not built: run `python paper_2510_11077_amd/build.py`")

# PyTorch ships its own HIP runtime; it is loaded first so that libargus
# binds to that same runtime (two runtimes in one process do not share
# devices, streams or allocations).
import torch  # noqa: E402,F401

_lib = C.CDLL(LIB_PATH)


class ArgusError(RuntimeError):
    pass


class _Desc(C.Structure):
    _fields_ = [("model", C.c_int32), ("n_psr", C.c_int32), ("toa_off", C.c_void_p),
                ("t", C.c_void_p), ("y", C.c_void_p), ("sigma", C.c_void_p),
                ("pos", C.c_void_p), ("fixed", C.c_void_p), ("free_mask", C.c_void_p),
                ("t_span", C.c_double), ("s_r", C.c_double), ("s_f", C.c_double),
                ("sigma_s", C.c_double), ("freq", C.c_void_p)]


_V = C.c_void_p
_lib.argus_last_error.restype = C.c_char_p
_lib.argus_dataset_create.argtypes = [C.POINTER(_Desc), C.POINTER(_V)]
_lib.argus_dataset_destroy.argtypes = [_V]
_lib.argus_dataset_n_params.argtypes = [_V, C.POINTER(C.c_int32)]
for _n in ("argus_loglike", "argus_loglike_terms", "argus_loglike_plain",
           "argus_loglike_noalloc"):
    getattr(_lib, _n).argtypes = [_V, _V, C.c_int64, _V, _V, _V]
_lib.argus_loglike_grad.argtypes = [_V, _V, C.c_int64, _V, _V, _V, _V]
_lib.argus_smooth.argtypes = [_V, _V, C.c_int64, _V, _V, _V, _V, _V]
_lib.argus_hmc_step.argtypes = [_V, C.c_int64, C.c_int32, _V, _V, _V, _V, _V, _V, _V, _V, _V,
                                _V, _V, _V]
_lib.argus_nuts_step.argtypes = [_V, C.c_int64, C.c_int32] + [_V] * 16
_lib.argus_tune_info.argtypes = [_V, C.c_int64, C.c_char_p, C.c_int32]
_lib.argus_filter_kernel_ms.argtypes = [_V, _V, C.c_int64, C.c_int32, C.POINTER(C.c_double), _V]
_lib.argus_fp64_rate.argtypes = [C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double), _V]
_lib.argus_mfma_rate.argtypes = [C.c_int32, C.c_int32, C.POINTER(C.c_double),
                                 C.POINTER(C.c_double), _V]
_lib.argus_mlp_create.argtypes = [C.c_int32, C.c_int32, C.c_int64, C.POINTER(_V)]
_lib.argus_mlp_destroy.argtypes = [_V]
_lib.argus_mlp_n_params.argtypes = [_V, C.POINTER(C.c_int64)]
_lib.argus_mlp_load.argtypes = [_V, _V, _V, _V, C.c_double, C.c_double, _V]
_lib.argus_mlp_load_affine.argtypes = [_V, _V, _V, _V, C.c_double, C.c_double, _V]
_lib.argus_surrogate_eval.argtypes = [_V, _V, C.c_int64, _V, _V]
_lib.argus_mlp_grad.argtypes = [_V, _V, _V, C.c_int64, _V, _V, _V]
_lib.argus_surrogate_train_step.argtypes = [_V, _V, _V, _V, _V, _V, C.c_int64, C.c_float,
                                            C.c_int64, _V, _V]
_lib.argus_surrogate_train_epoch.argtypes = [_V, _V, _V, _V, _V, _V, _V, C.c_int64, C.c_int64,
                                             C.c_float, C.c_int64, _V, _V]
_lib.argus_da_stage1.argtypes = [_V, _V, _V, _V, _V, _V, C.c_int64, C.c_int32, _V, _V, _V, _V]
_lib.argus_da_work_size.argtypes = [C.c_int64]
_lib.argus_da_work_size.restype = C.c_int64
_lib.argus_gather_rows.argtypes = [_V, _V, _V, C.c_int64, C.c_int32, _V, _V]
_lib.argus_da_stage2.argtypes = [_V, _V, C.c_int64, _V, _V, _V, _V, _V, _V, _V, _V, C.c_int32, _V]


def _check(rc: int):
    if rc != 0:
        raise ArgusError("libargus error %d: %s" % (rc, _lib.argus_last_error().decode()))


def _stream(stream=None) -> int:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def _dev_ptr(t, dtype, name):
    import torch
    if t is None:
        return None
    if not t.is_cuda:
        raise ArgusError("%s must be a device tensor" % name)
    if t.dtype != dtype:
        raise ArgusError("%s must be %s" % (name, dtype))
    if not t.is_contiguous():
        raise ArgusError("%s must be contiguous" % name)
    return t.data_ptr()


class Dataset:
    """A dataset handle. `d` is any object with the fields of the descriptor
    (model, n_psr, off, t, y, sigma, pos, t_span, s_r, s_f, sigma_s, truth as
    the fixed values, free as the free mask)."""

    def __init__(self, d):
        self.model = int(d.model)
        self.n_psr = int(d.n_psr)
        self.n_toa = int(np.asarray(d.off)[-1])
        self._keep = dict(
            off=np.ascontiguousarray(d.off, np.int64),
            t=np.ascontiguousarray(d.t, np.float64),
            y=np.ascontiguousarray(d.y, np.float64),
            sigma=np.ascontiguousarray(d.sigma, np.float64),
            pos=None if getattr(d, "pos", None) is None else np.ascontiguousarray(d.pos, np.float64),
            fixed=np.ascontiguousarray(d.truth, np.float64),
            free=None if getattr(d, "free", None) is None else np.ascontiguousarray(d.free, np.uint8),
            freq=None if getattr(d, "freq", None) is None else np.ascontiguousarray(d.freq, np.float64),
        )
        k = self._keep
        p = lambda a: None if a is None else a.ctypes.data
        desc = _Desc(self.model, self.n_psr, p(k["off"]), p(k["t"]), p(k["y"]), p(k["sigma"]),
                     p(k["pos"]) if self.model == M3_JOINT_HD else None, p(k["fixed"]), p(k["free"]),
                     float(d.t_span), float(d.s_r), float(d.s_f), float(d.sigma_s),
                     p(k["freq"]) if self.model == M4_PSR5_DM else None)
        h = _V()
        _check(_lib.argus_dataset_create(C.byref(desc), C.byref(h)))
        self._h = h
        D = C.c_int32()
        _check(_lib.argus_dataset_n_params(self._h, C.byref(D)))
        self.n_params = D.value

    def close(self):
        if getattr(self, "_h", None):
            _lib.argus_dataset_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------- calls
    def _theta(self, theta):
        import torch
        if theta.dim() != 2 or theta.shape[1] != self.n_params:
            raise ArgusError("theta must be [S, %d]" % self.n_params)
        return _dev_ptr(theta, torch.float64, "theta")

    def _outs(self, theta, out, status, want_status):
        import torch
        S = theta.shape[0]
        if out is None:
            out = torch.empty(S, dtype=torch.float64, device=theta.device)
        if status is None and want_status:
            status = torch.empty(S, dtype=torch.int32, device=theta.device)
        return out, status

    def loglike(self, theta, out=None, status=None, want_status=True, stream=None):
        """Batched logL: theta [S, D] float64 (device) -> (logl [S], status [S])."""
        import torch
        tp = self._theta(theta)
        out, status = self._outs(theta, out, status, want_status)
        _check(_lib.argus_loglike(self._h, tp, theta.shape[0], _dev_ptr(out, torch.float64, "out"),
                                  _dev_ptr(status, torch.int32, "status"), _stream(stream)))
        return out, status

    def loglike_noalloc(self, theta, out=None, status=None, want_status=True, stream=None):
        """argus_loglike_noalloc: the same outputs as loglike, from a call that
        allocates no device memory (models 1, 2, 4; S limited by the library's
        static scratch). Callers must supply out/status to allocate nothing
        on this side either."""
        import torch
        tp = self._theta(theta)
        out, status = self._outs(theta, out, status, want_status)
        _check(_lib.argus_loglike_noalloc(self._h, tp, theta.shape[0],
                                          _dev_ptr(out, torch.float64, "out"),
                                          _dev_ptr(status, torch.int32, "status"),
                                          _stream(stream)))
        return out, status

    def loglike_terms(self, theta, stream=None):
        """Per-pulsar terms [P, S] and status [S] (models 1, 2)."""
        import torch
        tp = self._theta(theta)
        S = theta.shape[0]
        terms = torch.empty((self.n_psr, S), dtype=torch.float64, device=theta.device)
        status = torch.empty(S, dtype=torch.int32, device=theta.device)
        _check(_lib.argus_loglike_terms(self._h, tp, S, terms.data_ptr(), status.data_ptr(),
                                        _stream(stream)))
        return terms, status

    def loglike_plain(self, theta, out=None, status=None, stream=None):
        """The plain one-launch-per-sample baseline filter (models 1, 2)."""
        import torch
        tp = self._theta(theta)
        out, status = self._outs(theta, out, status, True)
        _check(_lib.argus_loglike_plain(self._h, tp, theta.shape[0], out.data_ptr(),
                                        status.data_ptr(), _stream(stream)))
        return out, status

    def loglike_grad(self, theta, out=None, grad=None, status=None, stream=None):
        """logL [S] and d logL / d theta [S, D] (models 1, 2)."""
        import torch
        tp = self._theta(theta)
        out, status = self._outs(theta, out, status, True)
        if grad is None:
            grad = torch.empty_like(theta)
        _check(_lib.argus_loglike_grad(self._h, tp, theta.shape[0], out.data_ptr(),
                                       _dev_ptr(grad, torch.float64, "grad"), status.data_ptr(),
                                       _stream(stream)))
        return out, grad, status

    def smooth(self, theta, mean=None, var=None, want_var=True, stream=None):
        """Smoothed latent states (models 1, 2, 4): posterior mean and
        variance of each TOA's own pulsar state given all its TOAs, mean/var
        [N, nc, S] float64 (nc = 2 for model 1: r, f; 4 for model 2: r, f,
        a, g; 5 for model 4: r, f, a, g, m), plus logl [S] and status [S]."""
        import torch
        tp = self._theta(theta)
        S = theta.shape[0]
        nc = {M1_SPIN: 2, M4_PSR5_DM: 5}.get(self.model, 4)
        shape = (self.n_toa, nc, S)
        if mean is None:
            mean = torch.empty(shape, dtype=torch.float64, device=theta.device)
        if var is None and want_var:
            var = torch.empty(shape, dtype=torch.float64, device=theta.device)
        for name, t in (("mean", mean), ("var", var)):
            if t is not None and tuple(t.shape) != shape:
                raise ArgusError("%s must be %s" % (name, shape))
        out, status = self._outs(theta, None, None, True)
        _check(_lib.argus_smooth(self._h, tp, S, _dev_ptr(mean, torch.float64, "mean"),
                                 _dev_ptr(var, torch.float64, "var"), out.data_ptr(),
                                 status.data_ptr(), _stream(stream)))
        return mean, var, out, status

    def hmc_step(self, theta, logl, grad, eps, inv_mass, lo, hi, z, logu, n_leapfrog,
                 accepted, energy_err=None, stream=None):
        """One HMC transition per chain (rows of theta), in place on theta,
        logl, grad and accepted (see argus_hmc_step)."""
        import torch
        tp = self._theta(theta)
        S = theta.shape[0]
        f64 = torch.float64
        _check(_lib.argus_hmc_step(
            self._h, S, int(n_leapfrog), _dev_ptr(eps, f64, "eps"),
            _dev_ptr(inv_mass, f64, "inv_mass"), _dev_ptr(lo, f64, "lo"), _dev_ptr(hi, f64, "hi"),
            _dev_ptr(z, f64, "z"), _dev_ptr(logu, f64, "logu"), tp, _dev_ptr(logl, f64, "logl"),
            _dev_ptr(grad, f64, "grad"), _dev_ptr(accepted, torch.int32, "accepted"),
            _dev_ptr(energy_err, f64, "energy_err"), _stream(stream)))

    def nuts_step(self, theta, logl, grad, eps, inv_mass, lo, hi, z, dirs, u_top, u_sub,
                  max_depth, depth, n_leapfrog, divergent, accept_stat=None, stream=None):
        """One NUTS transition per chain, in place on theta, logl, grad (see
        argus_nuts_step)."""
        import torch
        tp = self._theta(theta)
        S = theta.shape[0]
        f64, i32 = torch.float64, torch.int32
        _check(_lib.argus_nuts_step(
            self._h, S, int(max_depth), _dev_ptr(eps, f64, "eps"),
            _dev_ptr(inv_mass, f64, "inv_mass"), _dev_ptr(lo, f64, "lo"), _dev_ptr(hi, f64, "hi"),
            _dev_ptr(z, f64, "z"), _dev_ptr(dirs, i32, "dirs"), _dev_ptr(u_top, f64, "u_top"),
            _dev_ptr(u_sub, f64, "u_sub"), tp, _dev_ptr(logl, f64, "logl"),
            _dev_ptr(grad, f64, "grad"), _dev_ptr(depth, i32, "depth"),
            _dev_ptr(n_leapfrog, i32, "n_leapfrog"), _dev_ptr(divergent, i32, "divergent"),
            _dev_ptr(accept_stat, f64, "accept_stat"), _stream(stream)))

    def filter_kernel_ms(self, theta, reps, stream=None) -> float:
        """Average duration (ms) of the tuned filter kernel alone over reps
        back-to-back launches (diagnostic; after a loglike call with this S)."""
        import torch
        ms = C.c_double()
        _check(_lib.argus_filter_kernel_ms(self._h, self._theta(theta), theta.shape[0], int(reps),
                                           C.byref(ms), _stream(stream)))
        return ms.value

    def tune_info(self, S: int) -> str:
        buf = C.create_string_buffer(4096)
        _check(_lib.argus_tune_info(self._h, S, buf, 4096))
        return buf.value.decode()


class MLP:
    """Surrogate network handle (argus_mlp_*). The packed FP32 master weights
    and Adam moments are torch tensors owned by this object."""

    def __init__(self, d_in, width=256, max_batch=4096, device="cuda"):
        import torch
        h = _V()
        _check(_lib.argus_mlp_create(d_in, width, max_batch, C.byref(h)))
        self._h = h
        n = C.c_int64()
        _check(_lib.argus_mlp_n_params(self._h, C.byref(n)))
        self.n_params, self.d_in, self.width, self.max_batch = n.value, d_in, width, max_batch
        self.master = torch.zeros(self.n_params, dtype=torch.float32, device=device)
        self.m = torch.zeros_like(self.master)
        self.v = torch.zeros_like(self.master)
        self.step = 0
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)

    def close(self):
        if getattr(self, "_h", None):
            _lib.argus_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load(self, master, in_lo, in_hi, out_mu, out_sd, stream=None):
        """Set the weights (packed FP32, any device tensor or array) and the
        input box / target standardisation."""
        import torch
        self.master.copy_(torch.as_tensor(master, dtype=torch.float32))
        self.m.zero_()
        self.v.zero_()
        self.step = 0
        self.in_lo = np.ascontiguousarray(in_lo, np.float64)
        self.in_hi = np.ascontiguousarray(in_hi, np.float64)
        self.out_mu, self.out_sd = float(out_mu), float(out_sd)
        _check(_lib.argus_mlp_load(self._h, self.master.data_ptr(), self.in_lo.ctypes.data,
                                   self.in_hi.ctypes.data, self.out_mu, self.out_sd,
                                   _stream(stream)))

    def load_affine(self, master, center, T, out_mu, out_sd, stream=None):
        """Set the weights and the affine input map x = T (theta - center)
        (T [d_in, d_in]) with the target standardisation."""
        import torch
        self.master.copy_(torch.as_tensor(master, dtype=torch.float32))
        self.m.zero_()
        self.v.zero_()
        self.step = 0
        self.in_center = np.ascontiguousarray(center, np.float64)
        self.in_T = np.ascontiguousarray(T, np.float64)
        if self.in_center.shape != (self.d_in,) or self.in_T.shape != (self.d_in, self.d_in):
            raise ArgusError("center must be [d_in] and T [d_in, d_in]")
        self.out_mu, self.out_sd = float(out_mu), float(out_sd)
        _check(_lib.argus_mlp_load_affine(self._h, self.master.data_ptr(),
                                          self.in_center.ctypes.data, self.in_T.ctypes.data,
                                          self.out_mu, self.out_sd, _stream(stream)))

    def eval(self, theta, out=None, stream=None):
        import torch
        theta = theta.contiguous()
        if out is None:
            out = torch.empty(theta.shape[0], dtype=torch.float64, device=theta.device)
        _check(_lib.argus_surrogate_eval(self._h, _dev_ptr(theta, torch.float64, "theta"),
                                         theta.shape[0], out.data_ptr(), _stream(stream)))
        return out

    def grad(self, theta, target, stream=None):
        import torch
        g = torch.empty(self.n_params, dtype=torch.float32, device=theta.device)
        _check(_lib.argus_mlp_grad(self._h, _dev_ptr(theta, torch.float64, "theta"),
                                   _dev_ptr(target, torch.float64, "target"), theta.shape[0],
                                   g.data_ptr(), self.loss.data_ptr(), _stream(stream)))
        return g, self.loss

    def train_epoch(self, theta, target, order, batch, lr, losses=None, stream=None):
        """len(order) // batch training steps in one library call; batch b
        uses rows order[b*batch:(b+1)*batch] of theta [N, d] / target [N]
        (device, float64); order: device int32. losses: optional device
        float32 [n_batches] for each batch's loss."""
        import torch
        n_batches = order.numel() // batch
        _check(_lib.argus_surrogate_train_epoch(
            self._h, self.master.data_ptr(), self.m.data_ptr(), self.v.data_ptr(),
            _dev_ptr(theta, torch.float64, "theta"), _dev_ptr(target, torch.float64, "target"),
            _dev_ptr(order, torch.int32, "order"), n_batches, batch, float(lr), self.step,
            _dev_ptr(losses, torch.float32, "losses"), _stream(stream)))
        self.step += n_batches
        return n_batches

    def train_step(self, theta, target, lr, stream=None):
        import torch
        self.step += 1
        _check(_lib.argus_surrogate_train_step(
            self._h, self.master.data_ptr(), self.m.data_ptr(), self.v.data_ptr(),
            _dev_ptr(theta, torch.float64, "theta"), _dev_ptr(target, torch.float64, "target"),
            theta.shape[0], float(lr), self.step, self.loss.data_ptr(), _stream(stream)))
        return self.loss


def da_stage1(theta_prop, lo, hi, lh_cur, lh_prop, logu1, idx, count, work, stream=None):
    Q, d = theta_prop.shape
    _check(_lib.argus_da_stage1(theta_prop.data_ptr(), lo.data_ptr(), hi.data_ptr(),
                                lh_cur.data_ptr(), lh_prop.data_ptr(), logu1.data_ptr(), Q, d,
                                idx.data_ptr(), count.data_ptr(), work.data_ptr(),
                                _stream(stream)))


def fp64_rate(waves_per_simd: int = 1, stream=None):
    """Sustained FP64 FMA rate (TFLOP/s) and mean shader clock (MHz) of the
    current device with every CU busy (argus_fp64_rate): the attainable
    ceiling for FP64-VALU kernels, next to the published peak."""
    tf, mhz = C.c_double(), C.c_double()
    _check(_lib.argus_fp64_rate(int(waves_per_simd), C.byref(tf), C.byref(mhz), _stream(stream)))
    return tf.value, mhz.value


def mfma_rate(kind: int, waves_per_simd: int = 1, stream=None):
    """Sustained matrix-core rate (TFLOP/s) and mean shader clock (MHz) with
    every CU busy (argus_mfma_rate): kind 1 FP64 16x16x4, kind 2 BF16
    32x32x16."""
    tf, mhz = C.c_double(), C.c_double()
    _check(_lib.argus_mfma_rate(int(kind), int(waves_per_simd), C.byref(tf), C.byref(mhz),
                                _stream(stream)))
    return tf.value, mhz.value


def da_work_size(Q: int) -> int:
    return int(_lib.argus_da_work_size(Q))


def gather_rows(src, idx, count, cap, dst, stream=None):
    _check(_lib.argus_gather_rows(src.data_ptr(), idx.data_ptr(), count.data_ptr(), cap,
                                  src.shape[1], dst.data_ptr(), _stream(stream)))


def da_stage2(idx, count, cap, ll_prop, lh_prop, logu2, theta_prop, theta_cur, ll_cur, lh_cur,
              acc, stream=None):
    _check(_lib.argus_da_stage2(idx.data_ptr(), count.data_ptr(), cap, ll_prop.data_ptr(),
                                lh_prop.data_ptr(), logu2.data_ptr(), theta_prop.data_ptr(),
                                theta_cur.data_ptr(), ll_cur.data_ptr(), lh_cur.data_ptr(),
                                acc.data_ptr(), theta_cur.shape[1], _stream(stream)))


class DelayedAcceptance:
    """Q parallel random-walk chains screened by the surrogate (stage 1) and
    judged by the exact filter (stage 2); every step runs in libargus
    kernels, this class only sequences them. Random numbers are drawn with
    torch and passed in. The survivor count is the only value read back per
    iteration (to size the exact evaluation)."""

    def __init__(self, ds, net, theta0, lo, hi, step_scale, seed=0):
        import torch
        self.ds, self.net = ds, net
        self.theta = theta0.clone().contiguous()
        self.Q, self.d = self.theta.shape
        dev = self.theta.device
        self.lo = torch.as_tensor(lo, dtype=torch.float64, device=dev)
        self.hi = torch.as_tensor(hi, dtype=torch.float64, device=dev)
        self.scale = torch.as_tensor(step_scale, dtype=torch.float64, device=dev)
        self.gen = torch.Generator(device=dev)
        self.gen.manual_seed(seed)
        self.ll, _ = ds.loglike(self.theta)
        self.ll = self.ll.clone()
        self.lh = net.eval(self.theta).clone()
        self.idx = torch.empty(self.Q, dtype=torch.int32, device=dev)
        self.count = torch.zeros(1, dtype=torch.int32, device=dev)
        self.work = torch.empty(da_work_size(self.Q), dtype=torch.int32, device=dev)
        self.acc = torch.zeros(self.Q, dtype=torch.int32, device=dev)
        # fixed buffers: the batched calls see the same pointers every step
        # (their captured graphs replay), sliced to the exact-evaluation size
        self.prop = torch.empty_like(self.theta)
        self.lh_prop = torch.empty_like(self.lh)
        self.sub = torch.empty_like(self.theta)
        self.ll_sub = torch.empty_like(self.ll)
        # exact-evaluation sizes are rounded up to a multiple of this, so only
        # a few sizes (each with its tuned workspace) ever occur
        self.gran = max(64, -(-self.Q // 32))
        self.n_exact = 0
        self.n_prop = 0

    def draws(self):
        import torch
        eps = torch.randn(self.theta.shape, dtype=torch.float64, device=self.theta.device,
                          generator=self.gen)
        # per-parameter scales [d], or a matrix L [d, d]: proposal covariance L L^T
        eps = eps @ self.scale.T if self.scale.dim() == 2 else eps * self.scale
        u = torch.rand((2, self.Q), dtype=torch.float64, device=self.theta.device,
                       generator=self.gen)
        return eps, torch.log(u[0]), torch.log(u[1])

    def step(self, eps=None, logu1=None, logu2=None, record=None):
        import torch
        if eps is None:
            eps, logu1, logu2 = self.draws()
        prop, lh_prop = self.prop, self.lh_prop
        torch.add(self.theta, eps, out=prop)
        self.net.eval(prop, out=lh_prop)
        da_stage1(prop, self.lo, self.hi, self.lh, lh_prop, logu1, self.idx, self.count,
                  self.work)
        n = int(self.count.item())
        self.n_prop += self.Q
        if record is not None:
            record.append(dict(prop=prop.clone(), lh_prop=lh_prop.clone(), lh_cur=self.lh.clone(),
                               ll_cur=self.ll.clone(), logu1=logu1.clone(), logu2=logu2.clone(),
                               theta=self.theta.clone(), n=n))
        if n == 0:
            return 0
        cap = min(-(-n // self.gran) * self.gran, self.Q)
        sub = self.sub[:cap]
        gather_rows(prop, self.idx, self.count, cap, sub)
        ll_prop, _ = self.ds.loglike(sub, out=self.ll_sub[:cap], want_status=False)
        self.n_exact += n
        da_stage2(self.idx, self.count, cap, ll_prop, lh_prop, logu2, prop, self.theta, self.ll,
                  self.lh, self.acc)
        return n


def pilot_posterior(ds, lo, hi, n_chains=4096, n_prior=65536, rounds=8, steps=40, keep=4,
                    seed=0):
    """Posterior draws without knowing the answer, by exact-likelihood
    Metropolis on the batched filter: n_prior draws uniform in the prior box
    [lo, hi] are evaluated in one batched call and the n_chains best start
    the chains; each round of `steps` random-walk Metropolis steps proposes
    from the Gaussian with covariance 2.38^2 / D times the ensemble's current
    covariance (adaptive Metropolis, Haario, Saksman & Tamminen 2001; Roberts,
    Gelman & Gilks 1997), a dense covariance that follows correlated
    parameters. Returns (theta [n_chains, D] final states, logl [n_chains],
    history [keep * steps * n_chains, D] states of the last `keep` rounds,
    their logL, the proposal factor L [D, D] (proposal L z, z standard
    normal), info). Sequencing only: every likelihood is argus_loglike."""
    import torch
    dev = "cuda"
    f64 = torch.float64
    lo_t = torch.as_tensor(lo, dtype=f64, device=dev)
    hi_t = torch.as_tensor(hi, dtype=f64, device=dev)
    D = lo_t.numel()
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    pr = lo_t + (hi_t - lo_t) * torch.rand((n_prior, D), dtype=f64, device=dev, generator=gen)
    lp, _ = ds.loglike(pr, want_status=False)
    best = torch.topk(torch.nan_to_num(lp, nan=-np.inf), n_chains).indices
    cur, llc = pr[best].contiguous(), lp[best].clone()
    prop = torch.empty_like(cur)
    llp = torch.empty_like(llc)
    hist, hll, acc_log = [], [], []
    jitter = np.diag((np.asarray(hi, np.float64) - np.asarray(lo, np.float64)) ** 2 * 1e-14)

    def proposal_factor(x):  # the D x D covariance work on the host
        C = np.cov(x.cpu().numpy(), rowvar=False) + jitter
        return torch.as_tensor(np.linalg.cholesky(C) * (2.38 / np.sqrt(D)), device=dev)

    for r in range(rounds):
        L = proposal_factor(cur)
        n_acc = torch.zeros((), dtype=torch.int64, device=dev)
        for _ in range(steps):
            z = torch.randn((n_chains, D), dtype=f64, device=dev, generator=gen)
            torch.addmm(cur, z, L.T, out=prop)
            ds.loglike(prop, out=llp, want_status=False)
            lu = torch.log(torch.rand(n_chains, dtype=f64, device=dev, generator=gen))
            ok = ((prop >= lo_t) & (prop <= hi_t)).all(1) & (lu < llp - llc)
            cur = torch.where(ok[:, None], prop, cur)
            llc = torch.where(ok, llp, llc)
            n_acc += ok.sum()
            if r >= rounds - keep:
                hist.append(cur)
                hll.append(llc)
        acc_log.append(int(n_acc.item()) / (steps * n_chains))
    L = proposal_factor(cur)
    info = {"prior_draws": n_prior, "chains": n_chains, "rounds": rounds,
            "steps_per_round": steps, "acceptance_per_round": acc_log}
    return cur, llc, torch.cat(hist), torch.cat(hll), L, info


def fit_surrogate(theta, logl, center, T, init_weights, width=256, batch=512, epochs=12,
                  lr=1e-3, floor=15.0, seed=0):
    """Trains the surrogate on exact (theta, logL) pairs with the library's
    training step: targets below max(logL) - floor are raised to that level
    (the network then only has to resolve the region a chain can move in;
    delayed acceptance stays exact whatever the surrogate says), standardised
    by their mean and standard deviation; input map x = T (theta - center);
    starting from init_weights (packed FP32); Adam with cosine-decayed
    learning rate over shuffled batches. Returns (net, info)."""
    import time as _time
    import torch
    n = theta.shape[0]
    y = torch.clamp(logl, min=float(logl.max().item()) - floor)
    mu, sd = float(y.mean().item()), float(y.std().item())
    net = MLP(theta.shape[1], width, batch)
    net.load_affine(init_weights, center, T, mu, sd)
    rng = np.random.default_rng(seed)
    perms = [torch.as_tensor(rng.permutation(n).astype(np.int32), device=theta.device)
             for _ in range(epochs)]
    losses = torch.empty(n // batch, dtype=torch.float32, device=theta.device)
    theta = theta.contiguous()
    steps = 0
    torch.cuda.synchronize()
    t0 = _time.perf_counter()
    for ep in range(epochs):
        lr_ep = lr * 0.5 * (1 + np.cos(np.pi * ep / epochs))
        steps += net.train_epoch(theta, y, perms[ep], batch, lr_ep, losses)
    torch.cuda.synchronize()
    info = {"samples": n, "epochs": epochs, "batch": batch, "steps": steps,
            "seconds": _time.perf_counter() - t0, "floor": floor,
            "final_loss": float(losses[-1].item())}
    return net, info


class HMC:
    """Batched Hamiltonian Monte Carlo on the gradient path: S chains (rows
    of theta0) with a uniform prior on [lo, hi], diagonal inverse mass
    inv_mass, step sizes eps (scalar or per chain) and n_leapfrog steps per
    transition. The random numbers (momentum draws, accept uniforms) come
    from a seeded device generator and are passed to argus_hmc_step."""

    def __init__(self, ds, theta0, lo, hi, eps, inv_mass, n_leapfrog, seed=0):
        import torch
        self.ds = ds
        dev = theta0.device
        f64 = torch.float64
        self.theta = theta0.to(f64).contiguous().clone()
        S, D = self.theta.shape
        self.lo = torch.as_tensor(lo, dtype=f64, device=dev).contiguous()
        self.hi = torch.as_tensor(hi, dtype=f64, device=dev).contiguous()
        self.inv_mass = torch.as_tensor(inv_mass, dtype=f64, device=dev).expand(D).contiguous()
        self.eps = torch.as_tensor(eps, dtype=f64, device=dev).expand(S).contiguous()
        self.n_leapfrog = int(n_leapfrog)
        self.logl, self.grad, st = ds.loglike_grad(self.theta)
        self.accepted = torch.zeros(S, dtype=torch.int32, device=dev)
        self.energy_err = torch.empty(S, dtype=f64, device=dev)
        self.z = torch.empty((S, D), dtype=f64, device=dev)
        self.u = torch.empty(S, dtype=f64, device=dev)
        self.gen = torch.Generator(device=dev)
        self.gen.manual_seed(seed)
        self.n_steps = 0

    def step(self, z=None, logu=None):
        """One transition of every chain; z, logu override the draws."""
        import torch
        if z is None:
            self.z.normal_(generator=self.gen)
            z = self.z
        if logu is None:
            self.u.uniform_(generator=self.gen)
            logu = torch.log(self.u)
        self.ds.hmc_step(self.theta, self.logl, self.grad, self.eps, self.inv_mass, self.lo,
                         self.hi, z, logu, self.n_leapfrog, self.accepted, self.energy_err)
        self.n_steps += 1

    def acceptance(self) -> float:
        return float(self.accepted.sum().item()) / max(1, self.n_steps * self.theta.shape[0])


class NUTS:
    """Batched No-U-Turn Sampler on the gradient path: S chains (rows of
    theta0), uniform prior on [lo, hi], diagonal inverse mass, step sizes
    eps (scalar or per chain), trees of at most max_depth doublings. The
    random numbers come from a seeded device generator and are passed to
    argus_nuts_step."""

    def __init__(self, ds, theta0, lo, hi, eps, inv_mass, max_depth=8, seed=0):
        import torch
        self.ds = ds
        dev = theta0.device
        f64, i32 = torch.float64, torch.int32
        self.theta = theta0.to(f64).contiguous().clone()
        S, D = self.theta.shape
        self.lo = torch.as_tensor(lo, dtype=f64, device=dev).contiguous()
        self.hi = torch.as_tensor(hi, dtype=f64, device=dev).contiguous()
        self.inv_mass = torch.as_tensor(inv_mass, dtype=f64, device=dev).expand(D).contiguous()
        self.eps = torch.as_tensor(eps, dtype=f64, device=dev).expand(S).contiguous()
        self.max_depth = int(max_depth)
        self.logl, self.grad, _ = ds.loglike_grad(self.theta)
        usz = 2 ** (self.max_depth - 1)
        self.z = torch.empty((S, D), dtype=f64, device=dev)
        self.dirs = torch.empty((S, self.max_depth), dtype=i32, device=dev)
        self.u_top = torch.empty((S, self.max_depth), dtype=f64, device=dev)
        self.u_sub = torch.empty((S, self.max_depth, usz), dtype=f64, device=dev)
        self.depth = torch.zeros(S, dtype=i32, device=dev)
        self.n_leapfrog = torch.zeros(S, dtype=i32, device=dev)
        self.divergent = torch.zeros(S, dtype=i32, device=dev)
        self.accept_stat = torch.zeros(S, dtype=f64, device=dev)
        self.gen = torch.Generator(device=dev)
        self.gen.manual_seed(seed)

    def step(self):
        """One transition of every chain."""
        self.z.normal_(generator=self.gen)
        self.u_top.uniform_(generator=self.gen)
        self.u_sub.uniform_(generator=self.gen)
        self.dirs.random_(0, 2, generator=self.gen)
        self.dirs.mul_(2).sub_(1)
        self.ds.nuts_step(self.theta, self.logl, self.grad, self.eps, self.inv_mass, self.lo,
                          self.hi, self.z, self.dirs, self.u_top, self.u_sub, self.max_depth,
                          self.depth, self.n_leapfrog, self.divergent, self.accept_stat)


def _make_loglike_fn():
    import torch

    class ArgusLogLike(torch.autograd.Function):
        """logL(theta) with argus_loglike_grad's gradient as its backward
        (the tangent sweep by default; the reverse-mode adjoint sweep with
        ARGUS_GRAD=adjoint)."""

        @staticmethod
        def forward(ctx, theta, ds):
            theta = theta.contiguous()
            logl, grad, _ = ds.loglike_grad(theta)
            ctx.save_for_backward(grad)
            return logl

        @staticmethod
        def backward(ctx, g):
            (grad,) = ctx.saved_tensors
            return g[:, None] * grad, None

    return ArgusLogLike


try:
    ArgusLogLike = _make_loglike_fn()
except ImportError:  # torch absent: the ctypes layer still loads
    ArgusLogLike = None
