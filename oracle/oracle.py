"""ctypes wrapper around ``u1ml_oracle.c`` (the FP64 CPU oracle).

TEST INFRASTRUCTURE ONLY: used by ``tests/``, by ``__graft_entry__.smoke()``
and by the CPU-baseline leg of ``bench.py``; the product library never imports
it.  Arrays cross the boundary as numpy FP64 arrays in the natural link order
``theta[t][z][y][x][mu]`` (mu = 0 is time).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

FIELD_MEMORY_LIMIT = 8 << 30  # bytes

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "u1ml_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-std=gnu11",
          "-shared", "-fPIC", "-Wall", "-Wno-unknown-pragmas"]


def build_oracle(force: bool = False) -> str:
    """Compile the oracle with gcc (no FMA contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build_oracle()
    lib = C.CDLL(_LIB)
    P = C.c_void_p
    dp = C.POINTER(C.c_double)
    ip = C.POINTER(C.c_int)
    u8p = C.POINTER(C.c_ubyte)
    u64p = C.POINTER(C.c_uint64)
    sig = {
        "or_create": (P, [C.c_int, C.c_int, C.c_double, C.c_double, C.c_uint64, C.c_int]),
        "or_destroy": (None, [P]),
        "or_volume": (C.c_long, [P]),
        "or_max_threads": (C.c_int, []),
        "or_set_threads": (None, [C.c_int]),
        "or_get_pass_id": (C.c_uint64, [P]),
        "or_set_pass_id": (None, [P, C.c_uint64]),
        "or_set_beta": (None, [P, C.c_double]),
        "or_get_links": (None, [P, dp]),
        "or_set_links": (None, [P, dp]),
        "or_staple": (None, [P, C.c_long, C.c_int, dp, dp]),
        "or_local_delta": (C.c_double, [P, C.c_long, C.c_int, C.c_double]),
        "or_total_action": (C.c_double, [P]),
        "or_class_pass": (None, [P, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_uint64, u8p]),
        "or_sweep": (C.c_long, [P, C.c_int, C.c_int, C.c_int, u8p]),
        "or_plaquette": (C.c_double, [P]),
        "or_polyakov": (None, [P, dp]),
        "or_plain_correlator": (None, [P, C.c_int, ip, dp]),
        "or_field_op": (C.c_double, [P, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int]),
        "or_field_means": (None, [P, dp]),
        "or_field2_means": (None, [P, dp]),
        "or_field_op2": (C.c_double, [P, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int]),
        "or_multilevel": (C.c_int, [P, C.c_int, ip, ip, C.c_int, C.c_int, C.c_int, ip, dp,
                                    C.c_int, ip, dp, u8p, C.c_long, C.POINTER(C.c_long), C.c_int]),
        "or_bessel_ratio": (C.c_double, [C.c_double]),
        "or_multihit_mean": (None, [P, C.c_long, dp]),
        "or_philox4x64_10": (None, [u64p, u64p, u64p]),
        "or_sincos": (None, [C.c_double, dp, dp]),
        "or_atan2": (C.c_double, [C.c_double, C.c_double]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int))


def _u8p(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_ubyte))


def philox4x64_10(ctr, key):
    lib = _load()
    c = np.asarray(ctr, dtype=np.uint64).copy()
    k = np.asarray(key, dtype=np.uint64).copy()
    out = np.zeros(4, dtype=np.uint64)
    p = C.POINTER(C.c_uint64)
    lib.or_philox4x64_10(c.ctypes.data_as(p), k.ctypes.data_as(p), out.ctypes.data_as(p))
    return out


def max_threads() -> int:
    return int(_load().or_max_threads())


def set_threads(n: int):
    """Threads of the oracle's OpenMP loops from now on (results do not depend on it)."""
    _load().or_set_threads(int(n))


def sincos(x: float):
    lib = _load()
    s, c = C.c_double(), C.c_double()
    lib.or_sincos(float(x), C.byref(s), C.byref(c))
    return s.value, c.value


def bessel_ratio(x: float) -> float:
    """I_1(x) / I_0(x)."""
    return _load().or_bessel_ratio(float(x))


def atan2(y: float, x: float) -> float:
    return _load().or_atan2(float(y), float(x))


class OracleLattice:
    """One FP64 lattice of the oracle."""

    def __init__(self, L: int, T: int, beta: float, seed: int, hot: bool = True, eps: float = 1.0):
        self._lib = _load()
        self._h = self._lib.or_create(L, T, float(beta), float(eps), int(seed), int(bool(hot)))
        if not self._h:
            raise ValueError("invalid lattice size (L, T must be even and >= 2)")
        self.L, self.T, self.beta, self.seed, self.eps = L, T, float(beta), int(seed), float(eps)
        self.V = L ** 3 * T

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.or_destroy(h)
            self._h = None

    # state ---------------------------------------------------------------
    @property
    def pass_id(self) -> int:
        return int(self._lib.or_get_pass_id(self._h))

    @pass_id.setter
    def pass_id(self, v: int):
        self._lib.or_set_pass_id(self._h, int(v))

    def set_beta(self, beta: float):
        self.beta = float(beta)
        self._lib.or_set_beta(self._h, self.beta)

    def get_links(self) -> np.ndarray:
        out = np.empty((self.T, self.L, self.L, self.L, 4), dtype=np.float64)
        self._lib.or_get_links(self._h, _dp(out))
        return out

    def set_links(self, th: np.ndarray):
        a = np.ascontiguousarray(th, dtype=np.float64).reshape(self.T, self.L, self.L, self.L, 4)
        self._lib.or_set_links(self._h, _dp(a))

    # local quantities ----------------------------------------------------
    def staple(self, n: int, mu: int):
        re, im = C.c_double(), C.c_double()
        self._lib.or_staple(self._h, int(n), int(mu), C.byref(re), C.byref(im))
        return re.value, im.value

    def multihit_mean(self, n: int) -> complex:
        """Conditional mean of exp(i theta_0) at canonical site n given all other links."""
        out = np.zeros(2)
        self._lib.or_multihit_mean(self._h, int(n), _dp(out))
        return complex(out[0], out[1])

    def local_delta(self, n: int, mu: int, v: float) -> float:
        return self._lib.or_local_delta(self._h, int(n), int(mu), float(v))

    def total_action(self) -> float:
        return self._lib.or_total_action(self._h)

    # updates -------------------------------------------------------------
    def class_pass(self, mu, parity, kind, n_hits=1, th_frozen=0, pass_id=0, log=None):
        self._lib.or_class_pass(self._h, mu, parity, kind, n_hits, th_frozen, int(pass_id), _u8p(log))

    def sweep(self, n_metro=1, n_or=3, th_frozen=0, want_log=False):
        log = np.zeros(8 * (self.V // 2) * n_metro, dtype=np.uint8) if want_log else None
        self._lib.or_sweep(self._h, n_metro, n_or, th_frozen, _u8p(log))
        return log

    # measurements --------------------------------------------------------
    def plaquette(self) -> float:
        return self._lib.or_plaquette(self._h)

    def polyakov(self):
        out = np.zeros(3)
        self._lib.or_polyakov(self._h, _dp(out))
        return out

    def plain_correlator(self, r_list):
        r = np.ascontiguousarray(r_list, dtype=np.int32)
        out = np.zeros(2 * len(r))
        self._lib.or_plain_correlator(self._h, len(r), _ip(r), _dp(out))
        return out[0::2] + 1j * out[1::2]

    def field_op(self, comp, t, x, y, z) -> float:
        return self._lib.or_field_op(self._h, comp, t, x, y, z)

    def field_means(self):
        out = np.zeros(6)
        self._lib.or_field_means(self._h, _dp(out))
        return out

    def field_op2(self, comp, t, x, y, z) -> float:
        """beta (1 - Re P) of the plaquette of component comp at (t, x, y, z)."""
        return self._lib.or_field_op2(self._h, comp, t, x, y, z)

    def field2_means(self):
        out = np.zeros(6)
        self._lib.or_field2_means(self._h, _dp(out))
        return out

    def multilevel(self, slab_sizes, n_sub, n_metro=1, n_or=3, r_list=(1,), rf_list=(),
                   log_cap=0, multihit=False, field_squared=False, symmetric=False):
        """Returns (C_ML[r] complex, field[rf][plane][comp][dy][dz] complex, log).
        symmetric: C_ML(r) averaged over the separations along +-x, +-y, +-z."""
        th = np.ascontiguousarray(slab_sizes, dtype=np.int32)
        ns = np.ascontiguousarray(n_sub, dtype=np.int32)
        r = np.ascontiguousarray(r_list, dtype=np.int32)
        rf = np.ascontiguousarray(rf_list if len(rf_list) else [0], dtype=np.int32)
        n_rf = len(rf_list)
        corr = np.zeros(2 * len(r))
        L = self.L
        field = np.zeros(max(n_rf, 1) * 2 * 6 * L * L * 2)
        log = np.zeros(max(log_cap, 1), dtype=np.uint8)
        # the field accumulators hold every (slab, source, r, plane, offset,
        # component) of a level: refuse sizes that would not fit in memory
        if n_rf:
            nslab = self.T // int(th[-1])
            need = 2 * nslab * L ** 3 * n_rf * 2 * L * L * 6 * 16
            if need > FIELD_MEMORY_LIMIT:
                raise MemoryError(f"oracle field accumulators need {need / 2**30:.1f} GiB "
                                  f"(limit {FIELD_MEMORY_LIMIT / 2**30:.0f} GiB); use a smaller lattice")
        used = C.c_long(0)
        rc = self._lib.or_multilevel(self._h, len(th), _ip(th), _ip(ns), n_metro, n_or, len(r), _ip(r),
                                     _dp(corr), n_rf, _ip(rf), _dp(field), _u8p(log) if log_cap else None,
                                     int(log_cap), C.byref(used),
                                     int(bool(multihit)) | (2 if field_squared else 0) | (4 if symmetric else 0))
        if rc != 0:
            raise ValueError("invalid multilevel arguments")
        f = field.reshape(max(n_rf, 1), 2, 6, L, L, 2)
        f = (f[..., 0] + 1j * f[..., 1])[:n_rf]
        return corr[0::2] + 1j * corr[1::2], f, log[: used.value]


def connected_profile(fields, corrs, omeans, r_list, rf_list):
    """Eq. (7) over an ensemble of multilevel runs:

        <O_c(d)>_{P*P} = mean <P*(0) P(r) O_c(d)> / mean <P*(0) P(r)> - mean <O_c>

    fields[k]: run k's field profile [n_rf][plane][comp][dy][dz] (complex),
    corrs[k]: its correlator over r_list, omeans[k]: the six lattice means of
    the inserted operators.  Means are plain averages over the runs; the
    quotient is the complex one.  Returns [n_rf][plane][comp][dy][dz]."""
    F = np.mean(np.asarray(fields), axis=0)
    Cm = np.mean(np.asarray(corrs), axis=0)
    O = np.mean(np.asarray(omeans, dtype=float), axis=0)
    r_list = list(r_list)
    out = np.empty_like(F)
    for f, r in enumerate(rf_list):
        out[f] = F[f] / Cm[r_list.index(r)] - O[None, :, None, None]
    return out
