"""ctypes binding of libatpool.so (the C ABI in include/at.h).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  Device arrays are torch tensors (PyTorch provides device memory and
the stream); host arrays are numpy.  The library must be built for gfx950 --
there is no fallback: a missing library raises at first use.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libatpool.so")

AT_OK, AT_E_INVAL, AT_E_STATE, AT_E_NOMEM, AT_E_OVERFLOW, AT_E_DEVICE, AT_E_BUDGET = 0, -1, -2, -3, -4, -5, -6
AT_F_SAT, AT_F_NEG, AT_F_FALLBACK, AT_F_SUPER = 1, 2, 4, 8
NOALLOC_MAX_PAIRS = 1 << 20           # AT_NOALLOC_MAX_PAIRS
AT_HIST_MAX_K = 1024                 # AT_HIST_MAX_K


class AtError(RuntimeError):
    def __init__(self, rc: int, where: str):
        super().__init__(f"{where}: {strerror(rc)} (rc={rc})")
        self.rc = rc


class Params(C.Structure):
    _fields_ = [("k", C.c_uint32), ("r", C.c_uint32), ("c", C.c_uint32), ("s", C.c_uint32),
                ("u", C.c_uint32), ("log2g", C.c_uint32), ("theta", C.c_double),
                ("seed", C.c_uint64), ("tuple_budget", C.c_uint64)]


# name -> (restype, argtypes); every symbol include/at.h declares
_vp = C.c_void_p
_u8p, _u32p, _u64p, _f64p, _f32p = (C.POINTER(C.c_uint8), C.POINTER(C.c_uint32), C.POINTER(C.c_uint64),
                                    C.POINTER(C.c_double), C.POINTER(C.c_float))
SIGNATURES = {
    "at_create": (C.c_int, [C.POINTER(Params), _vp, C.POINTER(_vp)]),
    "at_ingest_slice": (C.c_int, [_vp, _vp, _vp, C.c_uint64]),
    "at_ingest_slice_noalloc": (C.c_int, [_vp, _vp, _vp, C.c_uint64]),
    "at_close_slice": (C.c_int, [_vp, C.c_uint32]),
    "at_close_slice_multi": (C.c_int, [_vp, _u32p, C.c_uint32]),
    "at_select_window": (C.c_int, [_vp, C.c_uint32]),
    "at_close_slice_hist": (C.c_int, [_vp, C.c_uint32]),
    "at_requery_window": (C.c_int, [_vp, C.c_uint32]),
    "at_read_age_hist": (C.c_int, [_vp, _vp]),
    "at_estimate": (C.c_int, [_vp, _u32p, C.c_uint64, _f64p, _u8p]),
    "at_restore": (C.c_int, [_vp, _u32p, _f64p, _u8p, C.c_uint64, _u64p]),
    "at_destroy": (C.c_int, [_vp]),
    "at_strerror": (C.c_char_p, [C.c_int]),
    "at_pool_info": (C.c_int, [_vp, _u64p, _u64p]),
    "at_read_pool": (C.c_int, [_vp, _u8p]),
    "at_read_summary": (C.c_int, [_vp, _u32p, _u64p]),
    "at_clock": (C.c_int, [_vp, _u64p]),
    "at_constants": (C.c_int, [_vp, _u64p]),
    "at_estimate_detail": (C.c_int, [_vp, _u32p, C.c_uint64, _f64p, _u8p, _u32p]),
    "at_estimate_dev": (C.c_int, [_vp, _vp, C.c_uint64, _vp, _vp, _vp]),
    "at_tuple_count": (C.c_int, [_vp, _u64p]),
    "at_set_scan_mode": (C.c_int, [_vp, C.c_int]),
    "at_probe_scatter": (C.c_int, [_vp, C.c_uint64, _vp, _vp, C.c_uint64, C.c_uint32, _vp]),
    "at_cmp_create": (C.c_int, [C.POINTER(Params), C.c_int, _vp, C.POINTER(_vp)]),
    "at_cmp_destroy": (C.c_int, [_vp]),
    "at_cmp_info": (C.c_int, [_vp, _u64p]),
    "at_cmp_open_slice": (C.c_int, [_vp]),
    "at_cmp_ingest": (C.c_int, [_vp, _vp, _vp, C.c_uint64]),
    "at_cmp_close": (C.c_int, [_vp, C.c_uint32]),
    "at_cmp_read": (C.c_int, [_vp, _u32p, _u32p]),
    "at_features": (C.c_int, [_vp, _vp, C.c_uint64, _vp, _vp, _vp]),
    "at_mlp_create": (C.c_int, [_vp, C.POINTER(_vp)]),
    "at_mlp_destroy": (C.c_int, [_vp]),
    "at_mlp_set_params": (C.c_int, [_vp, _f32p]),
    "at_mlp_get_params": (C.c_int, [_vp, _f32p]),
    "at_mlp_forward": (C.c_int, [_vp, _vp, C.c_uint64, _vp]),
    "at_mlp_grad": (C.c_int, [_vp, _vp, _vp, C.c_uint64, _vp, _f32p]),
    "at_mlp_apply_grad": (C.c_int, [_vp, _vp, C.c_float]),
    "at_mlp_gather_batch": (C.c_int, [_vp, _vp, _vp, _vp, C.c_uint64, _vp, _vp]),
    "at_mlp_train_step": (C.c_int, [_vp, _vp, _vp, C.c_uint64, C.c_float, _f32p]),
    "at_estimate_learned": (C.c_int, [_vp, _vp, _u32p, C.c_uint64, _f64p, _u8p, _f64p]),
    "at_estimate_learned_dev": (C.c_int, [_vp, _vp, _vp, C.c_uint64, _vp, _vp, _vp]),
    "at_estimate_learned_begin": (C.c_int, [_vp, _vp, _u32p, C.c_uint64]),
    "at_estimate_learned_end": (C.c_int, [_vp, _f64p, _u8p, _f64p]),
}
MLP_NPARAM = 8385
FEATURES = 64


class ServeConfig(C.Structure):
    _fields_ = [("hbm_budget", C.c_uint64), ("max_links", C.c_uint32), ("cand_cap", C.c_uint32),
                ("watch_cap", C.c_uint32), ("r", C.c_uint32), ("c", C.c_uint32), ("s", C.c_uint32),
                ("u", C.c_uint32), ("log2g", C.c_uint32), ("theta", C.c_double)]


class ServeResult(C.Structure):
    _fields_ = [("link", C.c_uint32), ("kprime", C.c_uint32), ("slice", C.c_uint64), ("restore_rc", C.c_int32),
                ("n_cand", C.c_uint32), ("n_out", C.c_uint64), ("n_watch", C.c_uint32), ("pad", C.c_uint32),
                ("latency_ms", C.c_double), ("step_ms", C.c_double)]


SIGNATURES.update({
    "at_serve_create": (C.c_int, [C.POINTER(ServeConfig), C.POINTER(_vp)]),
    "at_serve_destroy": (C.c_int, [_vp]),
    "at_serve_set_mlp": (C.c_int, [_vp, _vp]),
    "at_serve_open_link": (C.c_int, [_vp, C.c_uint32, C.c_uint64, C.c_uint64, _u32p, C.POINTER(C.c_int)]),
    "at_serve_link_state": (C.c_int, [_vp, C.c_uint32, C.POINTER(C.c_int), _u64p, _u64p]),
    "at_serve_close_link": (C.c_int, [_vp, C.c_uint32]),
    "at_serve_set_watch": (C.c_int, [_vp, C.c_uint32, _u32p, C.c_uint32]),
    "at_serve_submit": (C.c_int, [_vp, C.c_uint32, _vp, _vp, C.c_uint64]),
    "at_serve_end_slice": (C.c_int, [_vp, C.c_uint32, C.c_uint32]),
    "at_serve_submit_last": (C.c_int, [_vp, C.c_uint32, _vp, _vp, C.c_uint64, C.c_uint32]),
    "at_serve_step": (C.c_int, [_vp, _u32p]),
    "at_serve_start": (C.c_int, [_vp]),
    "at_serve_stop": (C.c_int, [_vp]),
    "at_serve_next_result": (C.c_int, [_vp, C.POINTER(ServeResult), _u32p, _f64p, _f64p, _u8p, C.c_uint32,
                                       _f64p, _f64p, _u8p, C.c_uint32]),
    "at_serve_stats": (C.c_int, [_vp, _u64p]),
    "at_serve_read_pool": (C.c_int, [_vp, C.c_uint32, _u8p]),
    "at_serve_tiled_stats": (C.c_int, [_vp, _u64p, _u64p, _f64p, _u64p, _u64p]),
})

_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise ImportError(f"{path} is missing: build it with paper_1807_01527_amd/build.py "
                              "(hipcc --offload-arch=gfx950); there is no CPU fallback")
        lib = C.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def strerror(rc: int) -> str:
    try:
        return load().at_strerror(rc).decode()
    except ImportError:
        return str(rc)


def _p(a: np.ndarray, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def _dev_ptr(t) -> int:
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a device (cuda) tensor")
    if not t.is_contiguous():
        raise ValueError("device tensor must be contiguous")
    return t.data_ptr()


def _check(rc: int, where: str):
    if rc != AT_OK:
        raise AtError(rc, where)


def probe_scatter(dst_dev, a_dev, b_dev, n: int, r: int, stream=None):
    """Uniform random byte-store probe (see at_probe_scatter)."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    _check(load().at_probe_scatter(C.c_void_p(_dev_ptr(dst_dev)), dst_dev.numel() * dst_dev.element_size(),
                                   C.c_void_p(_dev_ptr(a_dev)), C.c_void_p(_dev_ptr(b_dev)), n, r,
                                   C.c_void_p(stream.cuda_stream)), "at_probe_scatter")


class AtPool:
    """One link: an ATVC pool in device memory, driven on a HIP stream."""

    def __init__(self, k: int, r: int, c: int, s: int, u: int, log2g: int, theta: float = 1024.0,
                 seed: int = 0, tuple_budget: int = 0, stream=None):
        import torch
        self.lib = load()
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        p = Params(k, r, c, s, u, log2g, theta, seed, tuple_budget)
        h = C.c_void_p()
        _check(self.lib.at_create(C.byref(p), C.c_void_p(stream.cuda_stream), C.byref(h)), "at_create")
        self.h = h
        self.k, self.r, self.c, self.s, self.u, self.log2g = k, r, c, s, u, log2g
        self.g = 1 << log2g
        self.theta = theta
        pb, na = C.c_uint64(), C.c_uint64()
        _check(self.lib.at_pool_info(self.h, C.byref(pb), C.byref(na)), "at_pool_info")
        self.pool_bytes, self.n_atv = int(pb.value), int(na.value)
        self.at_bytes = self.pool_bytes // (self.n_atv * self.g)   # 1, or 2 for k > 127
        self._pending_n = 0      # hosts of a pending estimate_learned_begin
        self._restore_out = None  # restore's output arrays, reused while cap stays the same

    @staticmethod
    def try_create(**kw) -> int:
        import torch
        lib = load()
        p = Params(kw["k"], kw["r"], kw["c"], kw["s"], kw["u"], kw["log2g"], kw.get("theta", 1024.0),
                   kw.get("seed", 0), kw.get("tuple_budget", 0))
        h = C.c_void_p()
        rc = lib.at_create(C.byref(p), C.c_void_p(torch.cuda.current_stream().cuda_stream), C.byref(h))
        if rc == AT_OK:
            lib.at_destroy(h)
        return rc

    def destroy(self):
        if getattr(self, "h", None):
            self.lib.at_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def _handle(self):
        if not self.h:
            raise AtError(AT_E_STATE, "handle destroyed")
        return self.h

    # ---- the six calls --------------------------------------------------
    def ingest(self, aip_dev, bip_dev, n: Optional[int] = None):
        if n is None:
            n = aip_dev.numel()
        if aip_dev.numel() < n or bip_dev.numel() < n:
            raise ValueError("n exceeds the device arrays")
        _check(self.lib.at_ingest_slice(self._handle(), C.c_void_p(_dev_ptr(aip_dev)),
                                        C.c_void_p(_dev_ptr(bip_dev)), n), "at_ingest_slice")

    def ingest_noalloc(self, aip_dev, bip_dev, n: Optional[int] = None) -> int:
        """at_ingest_slice_noalloc; returns its code (AT_E_INVAL above
        NOALLOC_MAX_PAIRS) instead of raising."""
        if n is None:
            n = aip_dev.numel()
        if aip_dev.numel() < n or bip_dev.numel() < n:
            raise ValueError("n exceeds the device arrays")
        return self.lib.at_ingest_slice_noalloc(self._handle(), C.c_void_p(_dev_ptr(aip_dev)),
                                                C.c_void_p(_dev_ptr(bip_dev)), n)

    def ingest_raw(self, aip_ptr: int, bip_ptr: int, n: int) -> int:
        return self.lib.at_ingest_slice(self._handle(), C.c_void_p(aip_ptr), C.c_void_p(bip_ptr), n)

    def close(self, kprime: Optional[int] = None):
        _check(self.lib.at_close_slice(self._handle(), self.k if kprime is None else kprime), "at_close_slice")

    def close_multi(self, kprimes):
        kp = np.ascontiguousarray(kprimes, np.uint32)
        _check(self.lib.at_close_slice_multi(self._handle(), _p(kp, C.c_uint32), kp.size), "at_close_slice_multi")

    def select_window(self, kprime: int):
        _check(self.lib.at_select_window(self._handle(), kprime), "at_select_window")

    def close_hist(self, kprime: Optional[int] = None):
        _check(self.lib.at_close_slice_hist(self._handle(), self.k if kprime is None else kprime),
               "at_close_slice_hist")

    def requery(self, kprime: int):
        _check(self.lib.at_requery_window(self._handle(), kprime), "at_requery_window")

    def read_age_hist(self) -> np.ndarray:
        out = np.zeros((self.n_atv, self.k), np.uint16)
        _check(self.lib.at_read_age_hist(self._handle(), out.ctypes.data_as(C.c_void_p)), "at_read_age_hist")
        return out

    def estimate(self, aip_host: np.ndarray) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
        aip = np.ascontiguousarray(aip_host, np.uint32)
        est = np.zeros(aip.size, np.float64)
        fl = np.zeros(aip.size, np.uint8)
        nat = np.zeros(aip.size, np.uint32)
        _check(self.lib.at_estimate_detail(self._handle(), _p(aip, C.c_uint32), aip.size, _p(est, C.c_double),
                                           _p(fl, C.c_uint8), _p(nat, C.c_uint32)), "at_estimate")
        return est, fl, nat

    def estimate_plain(self, aip_host: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
        aip = np.ascontiguousarray(aip_host, np.uint32)
        est = np.zeros(aip.size, np.float64)
        fl = np.zeros(aip.size, np.uint8)
        _check(self.lib.at_estimate(self._handle(), _p(aip, C.c_uint32), aip.size, _p(est, C.c_double),
                                    _p(fl, C.c_uint8)), "at_estimate")
        return est, fl

    def estimate_dev(self, aip_dev, est_dev=None, flags_dev=None, nat_dev=None):
        n = aip_dev.numel()
        ptr = lambda t: C.c_void_p(_dev_ptr(t)) if t is not None else C.c_void_p(0)  # noqa: E731
        _check(self.lib.at_estimate_dev(self._handle(), ptr(aip_dev), n, ptr(est_dev), ptr(flags_dev),
                                        ptr(nat_dev)), "at_estimate_dev")

    def restore(self, cap: int = 1 << 22):
        """Returns (rc, sips, est, flags, n_out); arrays are None unless rc == AT_OK."""
        size = max(cap, 1)
        if self._restore_out is None or self._restore_out[0].size != size:
            self._restore_out = (np.empty(size, np.uint32), np.empty(size, np.float64), np.empty(size, np.uint8))
        sip, est, fl = self._restore_out
        n = C.c_uint64()
        rc = self.lib.at_restore(self._handle(), _p(sip, C.c_uint32), _p(est, C.c_double), _p(fl, C.c_uint8),
                                 cap, C.byref(n))
        m = int(n.value)
        if rc == AT_OK:
            return rc, sip[:m].copy(), est[:m].copy(), fl[:m].copy(), m
        if rc in (AT_E_OVERFLOW, AT_E_BUDGET):
            return rc, None, None, None, m
        raise AtError(rc, "at_restore")

    # ---- introspection --------------------------------------------------
    def read_pool(self) -> np.ndarray:
        """AT values, uint8 (k <= 127) or uint16, ATV-major."""
        out = np.zeros(self.pool_bytes, np.uint8)
        _check(self.lib.at_read_pool(self._handle(), _p(out, C.c_uint8)), "at_read_pool")
        return out.view(np.uint16) if self.at_bytes == 2 else out

    def read_summary(self) -> Tuple[np.ndarray, np.ndarray]:
        w = np.zeros(self.n_atv, np.uint32)
        aat = np.zeros((1 << self.u) * self.r, np.uint64)
        _check(self.lib.at_read_summary(self._handle(), _p(w, C.c_uint32), _p(aat, C.c_uint64)),
               "at_read_summary")
        return w, aat

    def clock(self) -> dict:
        out = np.zeros(5, np.uint64)
        _check(self.lib.at_clock(self._handle(), _p(out, C.c_uint64)), "at_clock")
        return dict(zip(["t", "open", "queryable", "c0_query", "kq"], map(int, out)))

    def constants(self) -> dict:
        out = np.zeros(8, np.uint64)
        _check(self.lib.at_constants(self._handle(), _p(out, C.c_uint64)), "at_constants")
        return dict(zip(["p", "A", "Ainv", "alpha", "beta", "T", "W", "blk_a"], map(int, out)))

    def features(self, aip_dev, feat_dev, est_dev=None, flags_dev=None):
        n = aip_dev.numel()
        ptr = lambda t: C.c_void_p(_dev_ptr(t)) if t is not None else C.c_void_p(0)  # noqa: E731
        _check(self.lib.at_features(self._handle(), ptr(aip_dev), n, ptr(feat_dev), ptr(est_dev), ptr(flags_dev)),
               "at_features")

    def estimate_learned(self, mlp: "Mlp", aip_host: np.ndarray):
        """Returns (learned estimates, flags, plain estimates)."""
        aip = np.ascontiguousarray(aip_host, np.uint32)
        est = np.zeros(aip.size, np.float64)
        fl = np.zeros(aip.size, np.uint8)
        plain = np.zeros(aip.size, np.float64)
        _check(self.lib.at_estimate_learned(self._handle(), mlp._handle(), _p(aip, C.c_uint32), aip.size,
                                            _p(est, C.c_double), _p(fl, C.c_uint8), _p(plain, C.c_double)),
               "at_estimate_learned")
        return est, fl, plain

    def estimate_learned_begin(self, mlp: "Mlp", aip_host: np.ndarray):
        """Queue the learned estimates of the hosts; estimate_learned_end collects them."""
        aip = np.ascontiguousarray(aip_host, np.uint32)
        _check(self.lib.at_estimate_learned_begin(self._handle(), mlp._handle(), _p(aip, C.c_uint32), aip.size),
               "at_estimate_learned_begin")
        self._pending_n = aip.size

    def estimate_learned_end(self):
        """Wait for the estimates queued by estimate_learned_begin: (learned, flags, plain)."""
        n = self._pending_n
        est = np.empty(n, np.float64)
        fl = np.empty(n, np.uint8)
        plain = np.empty(n, np.float64)
        _check(self.lib.at_estimate_learned_end(self._handle(), _p(est, C.c_double), _p(fl, C.c_uint8),
                                                _p(plain, C.c_double)), "at_estimate_learned_end")
        return est, fl, plain

    def estimate_learned_dev(self, mlp: "Mlp", aip_dev, est_dev, flags_dev, plain_dev=None):
        ptr = lambda t: C.c_void_p(_dev_ptr(t)) if t is not None else C.c_void_p(0)  # noqa: E731
        _check(self.lib.at_estimate_learned_dev(self._handle(), mlp._handle(), ptr(aip_dev), aip_dev.numel(),
                                                ptr(est_dev), ptr(flags_dev), ptr(plain_dev)),
               "at_estimate_learned_dev")

    def set_scan_mode(self, mode: int):
        """0 automatic, 1 direct, 2 binned, 3 tiled (see at_set_scan_mode)."""
        _check(self.lib.at_set_scan_mode(self._handle(), mode), "at_set_scan_mode")

    def tuple_count(self) -> int:
        U = C.c_uint64()
        _check(self.lib.at_tuple_count(self._handle(), C.byref(U)), "at_tuple_count")
        return int(U.value)


class Mlp:
    """The learned-correction network (at_mlp_*): 64 -> 64 -> 64 -> 1."""

    def __init__(self, params: Optional[np.ndarray] = None, stream=None):
        import torch
        self.lib = load()
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        _check(self.lib.at_mlp_create(C.c_void_p(self.stream.cuda_stream), C.byref(h)), "at_mlp_create")
        self.h = h
        if params is not None:
            self.set_params(params)

    def _handle(self):
        if not self.h:
            raise AtError(AT_E_STATE, "network destroyed")
        return self.h

    def destroy(self):
        if getattr(self, "h", None):
            self.lib.at_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def set_params(self, params: np.ndarray):
        p = np.ascontiguousarray(params, np.float32)
        if p.size != MLP_NPARAM:
            raise ValueError("expected %d parameters" % MLP_NPARAM)
        _check(self.lib.at_mlp_set_params(self._handle(), _p(p, C.c_float)), "at_mlp_set_params")

    def get_params(self) -> np.ndarray:
        p = np.zeros(MLP_NPARAM, np.float32)
        _check(self.lib.at_mlp_get_params(self._handle(), _p(p, C.c_float)), "at_mlp_get_params")
        return p

    def forward(self, x_dev, y_dev):
        n = x_dev.shape[0]
        _check(self.lib.at_mlp_forward(self._handle(), C.c_void_p(_dev_ptr(x_dev)), n, C.c_void_p(_dev_ptr(y_dev))),
               "at_mlp_forward")

    def grad(self, x_dev, t_dev, grad_dev=None, want_loss: bool = True):
        loss = C.c_float()
        _check(self.lib.at_mlp_grad(self._handle(), C.c_void_p(_dev_ptr(x_dev)), C.c_void_p(_dev_ptr(t_dev)),
                                    x_dev.shape[0], C.c_void_p(_dev_ptr(grad_dev)) if grad_dev is not None else None,
                                    C.byref(loss) if want_loss else None), "at_mlp_grad")
        return float(loss.value) if want_loss else None

    def apply_grad(self, grad_dev, lr: float):
        _check(self.lib.at_mlp_apply_grad(self._handle(), C.c_void_p(_dev_ptr(grad_dev)), lr), "at_mlp_apply_grad")

    def gather_batch(self, x_dev, lnn_dev, idx_dev, xb_dev, tb_dev):
        """Rows idx of the features and their targets ln n - 16 f[61] (at_mlp_gather_batch)."""
        _check(self.lib.at_mlp_gather_batch(self._handle(), C.c_void_p(_dev_ptr(x_dev)), C.c_void_p(_dev_ptr(lnn_dev)),
                                            C.c_void_p(_dev_ptr(idx_dev)), idx_dev.numel(),
                                            C.c_void_p(_dev_ptr(xb_dev)), C.c_void_p(_dev_ptr(tb_dev))),
               "at_mlp_gather_batch")

    def train_step(self, x_dev, t_dev, lr: float, want_loss: bool = False):
        loss = C.c_float()
        _check(self.lib.at_mlp_train_step(self._handle(), C.c_void_p(_dev_ptr(x_dev)), C.c_void_p(_dev_ptr(t_dev)),
                                          x_dev.shape[0], lr, C.byref(loss) if want_loss else None),
               "at_mlp_train_step")
        return float(loss.value) if want_loss else None


class Server:
    """Streaming server (at_serve_*): many links, batched steps, one graph."""

    def __init__(self, hbm_budget: int, max_links: int, r: int, c: int, s: int, u: int, log2g: int,
                 theta: float = 1024.0, cand_cap: int = 2048, watch_cap: int = 256):
        self.lib = load()
        cfg = ServeConfig(hbm_budget, max_links, cand_cap, watch_cap, r, c, s, u, log2g, theta)
        h = C.c_void_p()
        _check(self.lib.at_serve_create(C.byref(cfg), C.byref(h)), "at_serve_create")
        self.h = h
        self.cand_cap, self.watch_cap = cand_cap, watch_cap
        self.pool_bytes = (1 << (c + u)) * r * (1 << log2g)
        self._keep = []

    def destroy(self):
        if getattr(self, "h", None):
            self.lib.at_serve_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def set_mlp(self, mlp: Optional["Mlp"]):
        _check(self.lib.at_serve_set_mlp(self.h, mlp._handle() if mlp is not None else None), "at_serve_set_mlp")
        self._mlp = mlp

    def open_link(self, k: int, seed: int, tuple_budget: int = 0) -> Tuple[int, bool]:
        lid = C.c_uint32()
        adm = C.c_int()
        _check(self.lib.at_serve_open_link(self.h, k, seed, tuple_budget, C.byref(lid), C.byref(adm)),
               "at_serve_open_link")
        return int(lid.value), bool(adm.value)

    def link_state(self, lid: int) -> Tuple[int, int, int]:
        st, t, pend = C.c_int(), C.c_uint64(), C.c_uint64()
        _check(self.lib.at_serve_link_state(self.h, lid, C.byref(st), C.byref(t), C.byref(pend)),
               "at_serve_link_state")
        return int(st.value), int(t.value), int(pend.value)

    def close_link(self, lid: int):
        _check(self.lib.at_serve_close_link(self.h, lid), "at_serve_close_link")

    def set_watch(self, lid: int, hosts: np.ndarray):
        hw = np.ascontiguousarray(hosts, np.uint32)
        _check(self.lib.at_serve_set_watch(self.h, lid, _p(hw, C.c_uint32), hw.size), "at_serve_set_watch")

    def submit(self, lid: int, aip_dev, bip_dev, n: Optional[int] = None) -> int:
        n = aip_dev.numel() if n is None else n
        return self.lib.at_serve_submit(self.h, lid, C.c_void_p(_dev_ptr(aip_dev)), C.c_void_p(_dev_ptr(bip_dev)), n)

    def end_slice(self, lid: int, kprime: int) -> int:
        return self.lib.at_serve_end_slice(self.h, lid, kprime)

    def submit_last(self, lid: int, aip_dev, bip_dev, kprime: int, n: Optional[int] = None) -> int:
        n = aip_dev.numel() if n is None else n
        return self.lib.at_serve_submit_last(self.h, lid, C.c_void_p(_dev_ptr(aip_dev)),
                                             C.c_void_p(_dev_ptr(bip_dev)), n, kprime)

    def step(self) -> int:
        n = C.c_uint32()
        _check(self.lib.at_serve_step(self.h, C.byref(n)), "at_serve_step")
        return int(n.value)

    def start(self):
        """Run steps on a native thread while work is queued."""
        _check(self.lib.at_serve_start(self.h), "at_serve_start")

    def stop(self):
        _check(self.lib.at_serve_stop(self.h), "at_serve_stop")

    def results(self):
        """Pop every ready result as dicts."""
        out = []
        cc, wc = self.cand_cap, self.watch_cap
        if getattr(self, "_rbuf", None) is None:   # staging reused across calls
            self._rbuf = (np.zeros(cc, np.uint32), np.zeros(cc), np.zeros(cc), np.zeros(cc, np.uint8),
                          np.zeros(max(wc, 1)), np.zeros(max(wc, 1)), np.zeros(max(wc, 1), np.uint8))
        cand, ce, cl, cf, wp, wl, wf = self._rbuf
        while True:
            r = ServeResult()
            rc = self.lib.at_serve_next_result(self.h, C.byref(r), _p(cand, C.c_uint32), _p(ce, C.c_double),
                                               _p(cl, C.c_double), _p(cf, C.c_uint8), cc, _p(wp, C.c_double),
                                               _p(wl, C.c_double), _p(wf, C.c_uint8), wc)
            if rc == AT_E_STATE:
                return out
            _check(rc, "at_serve_next_result")
            nc, nw = r.n_cand, r.n_watch
            out.append(dict(link=r.link, kprime=r.kprime, slice=r.slice, restore_rc=r.restore_rc, n_out=r.n_out,
                            cand=cand[:nc].copy(), cand_plain=ce[:nc].copy(), cand_learned=cl[:nc].copy(),
                            cand_flags=cf[:nc].copy(), watch_plain=wp[:nw].copy(), watch_learned=wl[:nw].copy(),
                            watch_flags=wf[:nw].copy(), latency_ms=r.latency_ms, step_ms=r.step_ms))

    def stats(self) -> dict:
        o = np.zeros(4, np.uint64)
        _check(self.lib.at_serve_stats(self.h, _p(o, C.c_uint64)), "at_serve_stats")
        return dict(steps=int(o[0]), pairs=int(o[1]), bytes=int(o[2]), waiting=int(o[3]))

    def read_pool(self, lid: int) -> np.ndarray:
        out = np.zeros(self.pool_bytes, np.uint8)
        _check(self.lib.at_serve_read_pool(self.h, lid, _p(out, C.c_uint8)), "at_serve_read_pool")
        return out

    def tiled_stats(self) -> dict:
        calls, pairs, ms, jobs, ahead = C.c_uint64(), C.c_uint64(), C.c_double(), C.c_uint64(), C.c_uint64()
        _check(self.lib.at_serve_tiled_stats(self.h, C.byref(calls), C.byref(pairs), C.byref(ms), C.byref(jobs),
                                             C.byref(ahead)), "at_serve_tiled_stats")
        return dict(calls=int(calls.value), jobs=int(jobs.value), pairs=int(pairs.value), device_ms=float(ms.value),
                    planned_ahead=int(ahead.value))


class AtCmp:
    """A packed comparator pool (at_cmp_*): ACE counters (kind "ace") or the
    asynchronous timestamps (kind "at"), each at its own width."""

    KINDS = {"ace": 1, "at": 2}

    def __init__(self, kind: str, k: int, r: int, c: int, s: int, u: int, log2g: int, theta: float = 1024.0,
                 seed: int = 0, stream=None):
        import torch
        self.lib = load()
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        p = Params(k, r, c, s, u, log2g, theta, seed, 0)
        h = C.c_void_p()
        _check(self.lib.at_cmp_create(C.byref(p), self.KINDS[kind], C.c_void_p(stream.cuda_stream), C.byref(h)),
               "at_cmp_create")
        self.h = h
        self.kind, self.k, self.g = kind, k, 1 << log2g
        self.n_atv = (1 << (c + u)) * r
        info = np.zeros(4, np.uint64)
        _check(self.lib.at_cmp_info(self.h, _p(info, C.c_uint64)), "at_cmp_info")
        self.bits, self.F, self.wv, self.n_words = (int(x) for x in info)

    def open_slice(self):
        _check(self.lib.at_cmp_open_slice(self.h), "at_cmp_open_slice")

    def ingest(self, aip_dev, bip_dev, n: Optional[int] = None):
        n = aip_dev.numel() if n is None else n
        _check(self.lib.at_cmp_ingest(self.h, C.c_void_p(_dev_ptr(aip_dev)), C.c_void_p(_dev_ptr(bip_dev)), n),
               "at_cmp_ingest")

    def close(self, kprime: Optional[int] = None):
        _check(self.lib.at_cmp_close(self.h, self.k if kprime is None else kprime), "at_cmp_close")

    def read_words(self) -> np.ndarray:
        out = np.zeros(self.n_words, np.uint32)
        _check(self.lib.at_cmp_read(self.h, _p(out, C.c_uint32), None), "at_cmp_read")
        return out

    def read_weights(self) -> np.ndarray:
        out = np.zeros(self.n_atv, np.uint32)
        _check(self.lib.at_cmp_read(self.h, None, _p(out, C.c_uint32)), "at_cmp_read")
        return out

    def unpack(self, words: np.ndarray) -> np.ndarray:
        """Field values per AT position (n_atv * g), from the packed layout
        at.h documents."""
        w = words.reshape(self.n_atv, self.wv).astype(np.uint64)
        mask = (1 << self.bits) - 1
        f = np.stack([(w >> np.uint64(e * self.bits)) & np.uint64(mask) for e in range(self.F)], axis=2)
        return f.reshape(self.n_atv, self.wv * self.F)[:, :self.g].reshape(-1).astype(np.uint32)

    def destroy(self):
        if getattr(self, "h", None):
            self.lib.at_cmp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
