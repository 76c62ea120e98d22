"""ctypes binding of the CPU oracle (liboracle.so).

TEST INFRASTRUCTURE ONLY: imported by the tests, the package smoke check and
the CPU-baseline leg of the benchmark, never by the product path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

OK, E_INVAL, E_STATE, E_NOMEM, E_OVERFLOW, E_BUDGET = 0, -1, -2, -3, -4, -6
F_SAT, F_NEG, F_SUPER = 1, 2, 8


class _Params(C.Structure):
    _fields_ = [("k", C.c_uint32), ("r", C.c_uint32), ("c", C.c_uint32), ("s", C.c_uint32),
                ("u", C.c_uint32), ("log2g", C.c_uint32), ("theta", C.c_double),
                ("seed", C.c_uint64), ("tuple_budget", C.c_uint64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b  # noqa
            _b.build()
        L = C.CDLL(LIB_PATH)
        u8p, u32p, u64p, f64p, f32p = (C.POINTER(C.c_uint8), C.POINTER(C.c_uint32),
                                      C.POINTER(C.c_uint64), C.POINTER(C.c_double),
                                      C.POINTER(C.c_float))
        vp = C.c_void_p
        sig = {
            "oat_create": (C.c_int, [C.POINTER(_Params), C.POINTER(vp)]),
            "oat_destroy": (None, [vp]),
            "oat_check_at": (C.c_int, [C.c_uint32] * 4),
            "oat_preserve_at": (C.c_uint32, [C.c_uint32] * 3),
            "oat_mangle": (C.c_uint32, [vp, C.c_uint32]),
            "oat_unmangle": (C.c_uint32, [vp, C.c_uint32]),
            "oat_rrh": (None, [vp, C.c_uint32, u32p, u32p]),
            "oat_bh": (C.c_uint32, [vp, C.c_uint32]),
            "oat_columns_of_L": (None, [vp, C.c_uint32, u32p]),
            "oat_tuple_to_L": (C.c_int, [vp, u32p, u32p]),
            "oat_tuple_dupcheck": (C.c_int, [vp, u32p]),
            "oat_block_of": (C.c_uint32, [vp, C.c_uint32]),
            "oat_ingest": (C.c_int, [vp, u32p, u32p, C.c_uint64]),
            "oat_close": (C.c_int, [vp, C.c_uint32]),
            "oat_requery": (C.c_int, [vp, C.c_uint32]),
            "oat_age_hist": (C.c_int, [vp, u32p]),
            "oat_ace_create": (C.c_int, [C.POINTER(_Params), C.POINTER(vp)]),
            "oat_ace_destroy": (None, [vp]),
            "oat_ace_ingest": (C.c_int, [vp, u32p, u32p, C.c_uint64]),
            "oat_ace_close": (C.c_int, [vp, C.c_uint32]),
            "oat_ace_bits": (C.c_uint32, [vp]),
            "oat_ace_counters": (vp, [vp]),
            "oat_ace_weights": (vp, [vp]),
            "oat_estimate": (C.c_int, [vp, u32p, C.c_uint64, f64p, u8p, u32p]),
            "oat_restore": (C.c_int, [vp, u32p, C.c_uint64, u64p]),
            "oat_tuple_count": (C.c_int, [vp, u64p]),
            "oat_features": (C.c_int, [vp, u32p, C.c_uint64, f32p]),
            "oat_pool_size": (C.c_uint64, [vp]),
            "oat_pool": (vp, [vp]),
            "oat_n_atv": (C.c_uint64, [vp]),
            "oat_weights": (vp, [vp]),
            "oat_aat": (vp, [vp]),
            "oat_super": (vp, [vp]),
            "oat_constants": (None, [vp, u64p]),
            "oat_clock": (None, [vp, u64p]),
            "oat_pin_bijection": (C.c_uint64, [vp, u32p]),
            "oat_pin_restore_bruteforce": (C.c_uint64, [vp, u8p, C.c_uint32, C.c_uint32, C.c_uint32,
                                                        C.c_uint32, u32p, C.c_uint64]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _p(a: np.ndarray, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def check_at(k: int, act: int, at: int, kprime: int) -> bool:
    return bool(lib().oat_check_at(k, act, at, kprime))


def preserve_at(k: int, act: int, at: int) -> int:
    return int(lib().oat_preserve_at(k, act, at))


class Oracle:
    """One ATV cube held by the oracle (one link)."""

    def __init__(self, k: int, r: int, c: int, s: int, u: int, log2g: int, theta: float = 1024.0,
                 seed: int = 0, tuple_budget: int = 0):
        self.params = dict(k=k, r=r, c=c, s=s, u=u, log2g=log2g, theta=theta, seed=seed,
                           tuple_budget=tuple_budget)
        p = _Params(k, r, c, s, u, log2g, theta, seed, tuple_budget)
        h = C.c_void_p()
        rc = lib().oat_create(C.byref(p), C.byref(h))
        if rc != OK:
            raise ValueError(f"oat_create rejected the parameters (rc={rc})")
        self.h = h
        self.k, self.r, self.c, self.s, self.u, self.log2g = k, r, c, s, u, log2g
        self.g = 1 << log2g
        self.theta = theta

    @staticmethod
    def try_create(**kw) -> int:
        p = _Params(kw["k"], kw["r"], kw["c"], kw["s"], kw["u"], kw["log2g"], kw.get("theta", 1024.0),
                    kw.get("seed", 0), kw.get("tuple_budget", 0))
        h = C.c_void_p()
        rc = lib().oat_create(C.byref(p), C.byref(h))
        if rc == OK:
            lib().oat_destroy(h)
        return rc

    def close_handle(self):
        if self.h:
            lib().oat_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close_handle()
        except Exception:
            pass

    # ---- primitives -----------------------------------------------------
    def mangle(self, a: int) -> int:
        return int(lib().oat_mangle(self.h, a))

    def unmangle(self, y: int) -> int:
        return int(lib().oat_unmangle(self.h, y))

    def rrh(self, a: int) -> Tuple[int, np.ndarray]:
        x = np.zeros(self.r, np.uint32)
        z = C.c_uint32()
        lib().oat_rrh(self.h, a, C.byref(z), _p(x, C.c_uint32))
        return int(z.value), x

    def bh(self, b: int) -> int:
        return int(lib().oat_bh(self.h, b))

    def columns_of_L(self, L: int) -> np.ndarray:
        x = np.zeros(self.r, np.uint32)
        lib().oat_columns_of_L(self.h, L, _p(x, C.c_uint32))
        return x

    def tuple_to_L(self, x) -> Optional[int]:
        x = np.ascontiguousarray(x, np.uint32)
        L = C.c_uint32()
        ok = lib().oat_tuple_to_L(self.h, _p(x, C.c_uint32), C.byref(L))
        return int(L.value) if ok else None

    def tuple_dupcheck(self, x) -> bool:
        x = np.ascontiguousarray(x, np.uint32)
        return bool(lib().oat_tuple_dupcheck(self.h, _p(x, C.c_uint32)))

    def block_of(self, i: int) -> int:
        return int(lib().oat_block_of(self.h, i))

    def constants(self) -> dict:
        out = np.zeros(8, np.uint64)
        lib().oat_constants(self.h, _p(out, C.c_uint64))
        keys = ["p", "A", "Ainv", "alpha", "beta", "T", "W", "blk_a"]
        return {k: int(v) for k, v in zip(keys, out)}

    def clock(self) -> dict:
        out = np.zeros(5, np.uint64)
        lib().oat_clock(self.h, _p(out, C.c_uint64))
        keys = ["t", "open", "queryable", "c0_query", "kq"]
        return {k: int(v) for k, v in zip(keys, out)}

    # ---- lifecycle ------------------------------------------------------
    def ingest(self, aip: np.ndarray, bip: np.ndarray) -> int:
        aip = np.ascontiguousarray(aip, np.uint32)
        bip = np.ascontiguousarray(bip, np.uint32)
        assert aip.shape == bip.shape
        return lib().oat_ingest(self.h, _p(aip, C.c_uint32), _p(bip, C.c_uint32), aip.size)

    def close(self, kprime: Optional[int] = None) -> int:
        return lib().oat_close(self.h, self.k if kprime is None else kprime)

    def requery(self, kprime: int) -> int:
        """Summarise the closed window again for another k' (clock unchanged)."""
        return lib().oat_requery(self.h, kprime)

    def age_hist(self) -> np.ndarray:
        """Per-ATV age histograms of the closed window: (n_atv, k) counts."""
        out = np.zeros((self.n_atv, self.k), np.uint32)
        rc = lib().oat_age_hist(self.h, _p(out, C.c_uint32))
        if rc:
            raise RuntimeError(f"oat_age_hist rc={rc}")
        return out

    def estimate(self, aip: np.ndarray):
        aip = np.ascontiguousarray(aip, np.uint32)
        est = np.zeros(aip.size, np.float64)
        fl = np.zeros(aip.size, np.uint8)
        nat = np.zeros(aip.size, np.uint32)
        rc = lib().oat_estimate(self.h, _p(aip, C.c_uint32), aip.size, _p(est, C.c_double),
                                _p(fl, C.c_uint8), _p(nat, C.c_uint32))
        if rc != OK:
            raise RuntimeError(f"oat_estimate rc={rc}")
        return est, fl, nat

    def tuple_count(self) -> int:
        U = C.c_uint64()
        rc = lib().oat_tuple_count(self.h, C.byref(U))
        if rc != OK:
            raise RuntimeError(f"oat_tuple_count rc={rc}")
        return int(U.value)

    def restore(self, cap: int = 1 << 22):
        """Returns (rc, sorted candidate array or None, n_out)."""
        out = np.zeros(max(cap, 1), np.uint32)
        n = C.c_uint64()
        rc = lib().oat_restore(self.h, _p(out, C.c_uint32), cap, C.byref(n))
        if rc == OK:
            return rc, out[: n.value].copy(), int(n.value)
        return rc, None, int(n.value)

    def features(self, aip: np.ndarray) -> np.ndarray:
        aip = np.ascontiguousarray(aip, np.uint32)
        f = np.zeros((aip.size, 64), np.float32)
        rc = lib().oat_features(self.h, _p(aip, C.c_uint32), aip.size, _p(f, C.c_float))
        if rc != OK:
            raise RuntimeError(f"oat_features rc={rc}")
        return f

    # ---- state ----------------------------------------------------------
    @property
    def pool_size(self) -> int:
        return int(lib().oat_pool_size(self.h))

    @property
    def n_atv(self) -> int:
        return int(lib().oat_n_atv(self.h))

    def pool(self) -> np.ndarray:
        """AT values (uint16, one per AT, ATV-major)."""
        ptr = lib().oat_pool(self.h)
        return np.ctypeslib.as_array(C.cast(ptr, C.POINTER(C.c_uint16)), (self.pool_size,)).copy()

    def weights(self) -> np.ndarray:
        ptr = lib().oat_weights(self.h)
        return np.ctypeslib.as_array(C.cast(ptr, C.POINTER(C.c_uint32)), (self.n_atv,)).copy()

    def aat(self) -> np.ndarray:
        ptr = lib().oat_aat(self.h)
        n = (1 << self.u) * self.r
        return np.ctypeslib.as_array(C.cast(ptr, C.POINTER(C.c_uint64)), (n,)).copy()

    def super_flags(self) -> np.ndarray:
        ptr = lib().oat_super(self.h)
        return np.ctypeslib.as_array(C.cast(ptr, C.POINTER(C.c_uint8)), (self.n_atv,)).copy()

    # ---- exhaustive pins ------------------------------------------------
    def pin_bijection(self) -> Tuple[int, int]:
        bad = C.c_uint32()
        n = lib().oat_pin_bijection(self.h, C.byref(bad))
        return int(n), int(bad.value)

    def pin_restore_bruteforce(self, cap: int = 1 << 22) -> Tuple[int, np.ndarray]:
        sup = np.ascontiguousarray(self.super_flags())
        out = np.zeros(max(cap, 1), np.uint32)
        n = lib().oat_pin_restore_bruteforce(self.h, _p(sup, C.c_uint8), self.r, self.c, self.s,
                                             self.u, _p(out, C.c_uint32), cap)
        return int(n), np.sort(out[: min(n, cap)])


class AceOracle:
    """ACE, the aging-counter comparator (Section 2.3), on the cube and hashes
    of an Oracle with the same parameters: ceil(log2(k+1))-bit counters set to
    their largest value, decreased at every slice after the first."""

    def __init__(self, k: int, r: int, c: int, s: int, u: int, log2g: int, theta: float = 1024.0,
                 seed: int = 0, tuple_budget: int = 0):
        p = _Params(k, r, c, s, u, log2g, theta, seed, tuple_budget)
        h = C.c_void_p()
        rc = lib().oat_ace_create(C.byref(p), C.byref(h))
        if rc != OK:
            raise ValueError(f"oat_ace_create rejected the parameters (rc={rc})")
        self.h = h
        self.k, self.r, self.c, self.u = k, r, c, u
        self.g = 1 << log2g
        self.n_atv = (1 << (c + u)) * r
        self.bits = int(lib().oat_ace_bits(h))
        self.cmax = (1 << self.bits) - 1

    def ingest(self, aip: np.ndarray, bip: np.ndarray) -> int:
        aip = np.ascontiguousarray(aip, np.uint32)
        bip = np.ascontiguousarray(bip, np.uint32)
        return lib().oat_ace_ingest(self.h, _p(aip, C.c_uint32), _p(bip, C.c_uint32), aip.size)

    def close(self, kprime: Optional[int] = None) -> int:
        return lib().oat_ace_close(self.h, self.k if kprime is None else kprime)

    def counters(self) -> np.ndarray:
        ptr = lib().oat_ace_counters(self.h)
        n = self.n_atv * self.g
        return np.ctypeslib.as_array(C.cast(ptr, C.POINTER(C.c_uint16)), (n,)).copy()

    def weights(self) -> np.ndarray:
        ptr = lib().oat_ace_weights(self.h)
        return np.ctypeslib.as_array(C.cast(ptr, C.POINTER(C.c_uint32)), (self.n_atv,)).copy()

    def __del__(self):
        try:
            if self.h:
                lib().oat_ace_destroy(self.h)
                self.h = None
        except Exception:
            pass
