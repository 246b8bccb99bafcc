"""Thin Python binding of the u1ml C ABI (``include/u1ml.h``).

Argument marshalling only: every step of the method runs in the HIP kernels of
``libu1ml.so``.  PyTorch supplies the device memory for the links and the HIP
stream work is queued on.  The functions carry the C names without the
``u1ml_`` prefix; a :class:`Lattice` / :class:`Batch` holds the handle.

There is no fallback: if the library is missing or no GPU is visible the calls
raise.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libu1ml.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "u1ml.h")

OK, EINVAL, ENOMEM, EDEVICE, ESTATE, EIO = 0, -1, -2, -3, -4, -5
COLD, HOT = 0, 1
FP64, FP32 = 0, 1
MAX_LEVELS = 3
MAX_FIELD_R = 32
FIELD_NAMES = ("Ex", "Ey", "Ez", "Bx", "By", "Bz")


class U1MLError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"u1ml error {code}: {msg}")
        self.code = code


class Options(C.Structure):
    _fields_ = [("start", C.c_int), ("precision", C.c_int), ("eps", C.c_double), ("stream", C.c_void_p),
                ("dev_buf", C.c_void_p), ("dev_bytes", C.c_size_t), ("block", C.c_int), ("no_graphs", C.c_int)]


class Observables(C.Structure):
    _fields_ = [("plaquette", C.c_double), ("poly_re", C.c_double), ("poly_im", C.c_double),
                ("poly_abs", C.c_double), ("field_mean", C.c_double * 6),
                ("field2_mean", C.c_double * 6)]

    def as_dict(self):
        return {"plaquette": self.plaquette, "poly": complex(self.poly_re, self.poly_im),
                "poly_abs": self.poly_abs, "field_mean": list(self.field_mean),
                "field2_mean": list(self.field2_mean)}


class Tuning(C.Structure):
    """u1ml_tuning: launch shapes of the kernels (results do not depend on them)."""
    _fields_ = [("pass_block", C.c_int), ("pass_xcd_map", C.c_int), ("sample_block", C.c_int),
                ("fold_threads", C.c_int), ("field_w_planes", C.c_int), ("field_o_planes", C.c_int),
                ("field_zcon_threads", C.c_int), ("fold_stage", C.c_int)]

    def as_dict(self):
        return {name: int(getattr(self, name)) for name, _ in self._fields_}


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libu1ml.so (built by ``paper_1208_0166_amd.build``); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1208_0166_amd.build`")
    # torch first: its HIP runtime (soname libamdhip64.so.7) is then the one the
    # library binds to, so the process holds a single runtime and torch device
    # buffers and streams are valid in library calls.
    import torch  # noqa: F401
    lib = C.CDLL(path)
    P, I, D, U64, SZ = C.c_void_p, C.c_int, C.c_double, C.c_uint64, C.c_size_t
    ip, dp = C.POINTER(C.c_int), C.POINTER(C.c_double)
    sig = {
        "u1ml_default_options": (None, [C.POINTER(Options)]),
        "u1ml_link_bytes": (SZ, [I, I, I]),
        "u1ml_workspace_bytes": (SZ, [I, I, I, I, ip, ip, I, I, C.c_uint]),
        "u1ml_device_bytes": (SZ, [P]),
        "u1ml_init_lattice": (I, [I, I, D, U64, C.POINTER(Options), C.POINTER(P)]),
        "u1ml_sweep": (I, [P, I, I]),
        "u1ml_multilevel": (I, [P, I, ip, ip, I, I, I, ip, I, ip]),
        "u1ml_measure": (I, [P, C.POINTER(Observables), dp, dp]),
        "u1ml_multilevel_noalloc": (I, [P, I, ip, ip, I, I, I, ip, P]),
        "u1ml_plain_correlator": (I, [P, I, ip, dp]),
        "u1ml_ensemble_reset": (I, [P]),
        "u1ml_ensemble_add": (I, [P]),
        "u1ml_ensemble_info": (I, [P, ip, ip, ip]),
        "u1ml_ensemble_read": (I, [P, dp, dp, dp]),
        "u1ml_batch_ensemble_reset": (I, [P]),
        "u1ml_batch_ensemble_add": (I, [P]),
        "u1ml_batch_ensemble_info": (I, [P, I, ip, ip, ip]),
        "u1ml_batch_ensemble_read": (I, [P, I, dp, dp, dp]),
        "u1ml_get_links": (I, [P, dp]),
        "u1ml_set_links": (I, [P, dp]),
        "u1ml_get_pass_id": (I, [P, C.POINTER(U64)]),
        "u1ml_set_pass_id": (I, [P, U64]),
        "u1ml_set_debug": (I, [P, C.c_uint, SZ]),
        "u1ml_set_estimator": (I, [P, C.c_uint]),
        "u1ml_batch_set_estimator": (I, [P, C.c_uint]),
        "u1ml_get_accept_log": (I, [P, C.POINTER(C.c_uint8), SZ, C.POINTER(SZ)]),
        "u1ml_save": (I, [P, C.c_char_p]),
        "u1ml_load": (I, [P, C.c_char_p]),
        "u1ml_synchronize": (I, [P]),
        "u1ml_destroy": (None, [P]),
        "u1ml_batch_create": (I, [I, ip, ip, dp, C.POINTER(U64), C.POINTER(Options), C.POINTER(P)]),
        "u1ml_batch_sweep": (I, [P, I, I]),
        "u1ml_batch_multilevel": (I, [P, I, ip, ip, I, I, I, ip, I, ip]),
        "u1ml_batch_cycle": (I, [P, I, I, I, I, I, I]),
        "u1ml_batch_measure": (I, [P, I, C.POINTER(Observables), dp, dp]),
        "u1ml_batch_get_links": (I, [P, I, dp]),
        "u1ml_batch_set_links": (I, [P, I, dp]),
        "u1ml_batch_get_pass_id": (I, [P, I, C.POINTER(U64)]),
        "u1ml_batch_set_pass_id": (I, [P, I, U64]),
        "u1ml_batch_save": (I, [P, C.c_char_p]),
        "u1ml_batch_load": (I, [P, C.c_char_p]),
        "u1ml_batch_synchronize": (I, [P]),
        "u1ml_batch_destroy": (None, [P]),
        "u1ml_autotune": (I, [P, ip]),
        "u1ml_get_tuning": (I, [P, C.POINTER(Tuning)]),
        "u1ml_set_tuning": (I, [P, C.POINTER(Tuning)]),
        "u1ml_batch_get_tuning": (I, [P, C.POINTER(Tuning)]),
        "u1ml_batch_set_tuning": (I, [P, C.POINTER(Tuning)]),
        "u1ml_batch_autotune": (I, [P, I, ip, ip, I, ip, I, ip, C.POINTER(Tuning)]),
        "u1ml_profile_sweeps": (I, [P, I, I, I, dp]),
        "u1ml_batch_profile_sweeps": (I, [P, I, I, I, dp]),
        "u1ml_stream_bandwidth": (I, [I, SZ, I, dp]),
        "u1ml_strerror": (C.c_char_p, [I]),
        "u1ml_last_error": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def header_functions(path: str = HEADER_PATH) -> list[str]:
    """Names of the functions declared in include/u1ml.h."""
    text = open(path).read()
    return sorted(set(re.findall(r"\b(u1ml_[a-z_0-9]+)\s*\(", text)))


def _check(rc: int):
    if rc != OK:
        lib = load_library()
        raise U1MLError(rc, f"{lib.u1ml_strerror(rc).decode()}: {lib.u1ml_last_error().decode()}")


def _ints(v):
    a = np.ascontiguousarray(v, dtype=np.int32)
    return a, a.ctypes.data_as(C.POINTER(C.c_int))


def link_bytes(L: int, T: int, precision: int = FP64) -> int:
    return int(load_library().u1ml_link_bytes(L, T, precision))


def default_options() -> Options:
    o = Options()
    load_library().u1ml_default_options(C.byref(o))
    return o


def _torch_stream(stream):
    import torch
    if stream is None:
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return C.c_void_p(int(stream))


class Lattice:
    """One lattice: wraps a ``u1ml_lattice*``."""

    def __init__(self, handle, L, T, beta, seed, precision, keepalive=None):
        self._h = handle
        self.L, self.T, self.beta, self.seed, self.precision = L, T, beta, seed, precision
        self.V = L ** 3 * T
        self._keep = keepalive
        self._n_r = 0
        self._n_rf = 0
        # bound now: module globals may already be gone when __del__ runs at exit
        self._destroy = load_library().u1ml_destroy

    def __del__(self):
        self.close()

    def close(self):
        if getattr(self, "_h", None):
            self._destroy(self._h)
            self._h = None
            self._keep = None

    @property
    def handle(self):
        return self._h


def init_lattice(L: int, T: int, beta: float, seed: int, *, start: int = HOT, precision: int = FP64,
                 eps: float = 1.0, block: int = 0, stream=None, torch_buffer: bool = True,
                 graphs: bool = True) -> Lattice:
    """u1ml_init_lattice; the link storage is a torch device tensor unless torch_buffer=False."""
    lib = load_library()
    o = default_options()
    o.start, o.precision, o.eps, o.block = start, precision, float(eps), block
    o.no_graphs = 0 if graphs else 1
    keep = None
    if torch_buffer:
        import torch
        nbytes = link_bytes(L, T, precision)
        if nbytes == 0:
            raise U1MLError(EINVAL, "invalid lattice size")
        keep = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        o.dev_buf, o.dev_bytes = keep.data_ptr(), nbytes
        o.stream = _torch_stream(stream)
    elif stream is not None:
        o.stream = C.c_void_p(int(stream))
    h = C.c_void_p()
    _check(lib.u1ml_init_lattice(L, T, float(beta), int(seed), C.byref(o), C.byref(h)))
    return Lattice(h, L, T, float(beta), int(seed), precision, keep)


def sweep(lat: Lattice, n_metro: int = 1, n_or: int = 3):
    _check(load_library().u1ml_sweep(lat.handle, n_metro, n_or))


def multilevel(lat: Lattice, slab_sizes, n_sub, n_metro: int = 1, n_or: int = 3, r_list=(1,), rf_list=()):
    th, thp = _ints(slab_sizes)
    ns, nsp = _ints(n_sub)
    r, rp = _ints(r_list)
    rf, rfp = _ints(rf_list if len(rf_list) else [0])
    _check(load_library().u1ml_multilevel(lat.handle, len(th), thp, nsp, n_metro, n_or, len(r), rp,
                                          len(rf_list), rfp if len(rf_list) else None))
    lat._n_r, lat._n_rf = len(r), len(rf_list)


def measure(lat: Lattice, observables: bool = True, correlator: bool = False, field_profile: bool = False):
    """Returns (obs dict or None, correlator complex[n_r] or None,
    field complex[n_rf][2][6][L][L] or None)."""
    obs = Observables() if observables else None
    corr = np.zeros(2 * lat._n_r) if correlator else None
    fp = np.zeros(lat._n_rf * 2 * 6 * lat.L * lat.L * 2) if field_profile else None
    _check(load_library().u1ml_measure(
        lat.handle, C.byref(obs) if obs is not None else None,
        corr.ctypes.data_as(C.POINTER(C.c_double)) if corr is not None else None,
        fp.ctypes.data_as(C.POINTER(C.c_double)) if fp is not None else None))
    c = corr[0::2] + 1j * corr[1::2] if corr is not None else None
    f = None
    if fp is not None:
        f = fp.reshape(lat._n_rf, 2, 6, lat.L, lat.L, 2)
        f = f[..., 0] + 1j * f[..., 1]
    return (obs.as_dict() if obs is not None else None), c, f


def multilevel_noalloc(lat: Lattice, slab_sizes, n_sub, n_metro: int = 1, n_or: int = 3, r_list=(1,), out=None):
    """u1ml_multilevel_noalloc: the multilevel correlator with the library's
    static device workspace; ``out`` is a caller-owned float64 CUDA tensor of
    2 * len(r_list) values, filled with (Re, Im) of C_ML(r).  Returns ``out``."""
    import torch
    th, thp = _ints(slab_sizes)
    ns, nsp = _ints(n_sub)
    r, rp = _ints(r_list)
    if out is None or not out.is_cuda or out.dtype != torch.float64 or out.numel() < 2 * len(r):
        raise U1MLError(EINVAL, "out must be a float64 CUDA tensor of 2 * len(r_list) values")
    _check(load_library().u1ml_multilevel_noalloc(lat.handle, len(th), thp, nsp, n_metro, n_or, len(r), rp,
                                                  C.c_void_p(out.data_ptr())))
    return out


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def _ensemble_read(info, read, L, correlator, field_profile, connected):
    n, nr, nrf = C.c_int(), C.c_int(), C.c_int()
    _check(info(C.byref(n), C.byref(nr), C.byref(nrf)))
    corr = np.zeros(2 * nr.value) if correlator else None
    fp = np.zeros(nrf.value * 2 * 6 * L * L * 2) if field_profile else None
    cn = np.zeros(nrf.value * 2 * 6 * L * L * 2) if connected else None
    _check(read(_dptr(corr), _dptr(fp), _dptr(cn)))

    def cplx(a, shape):
        if a is None:
            return None
        a = a.reshape(*shape, 2)
        return a[..., 0] + 1j * a[..., 1]
    fshape = (nrf.value, 2, 6, L, L)
    return n.value, cplx(corr, (nr.value,)), cplx(fp, fshape), cplx(cn, fshape)


def ensemble_reset(lat: Lattice):
    _check(load_library().u1ml_ensemble_reset(lat.handle))


def ensemble_add(lat: Lattice):
    _check(load_library().u1ml_ensemble_add(lat.handle))


def ensemble_read(lat: Lattice, correlator: bool = True, field_profile: bool = False, connected: bool = False):
    """Returns (n_runs, mean C complex[n_r] or None, mean field complex[n_rf][2][6][L][L]
    or None, connected profile of Eq. (7), same shape, or None)."""
    lib = load_library()
    return _ensemble_read(lambda *a: lib.u1ml_ensemble_info(lat.handle, *a),
                          lambda *a: lib.u1ml_ensemble_read(lat.handle, *a), lat.L, correlator, field_profile,
                          connected)


def workspace_bytes(L: int, T: int, slab_sizes, n_sub, n_r: int, n_rf: int = 0, multihit: bool = False,
                    field_squared: bool = False, symmetric: bool = False, precision: int = FP64) -> int:
    """Device bytes of a multilevel run's workspace (u1ml_workspace_bytes)."""
    th, thp = _ints(slab_sizes)
    ns, nsp = _ints(n_sub)
    return load_library().u1ml_workspace_bytes(L, T, precision, len(th), thp, nsp, n_r, n_rf,
                                               _estimator_flags(multihit, field_squared, symmetric))


def device_bytes(lat: Lattice) -> int:
    return load_library().u1ml_device_bytes(lat.handle)


def plain_correlator(lat: Lattice, r_list):
    r, rp = _ints(r_list)
    out = np.zeros(2 * len(r))
    _check(load_library().u1ml_plain_correlator(lat.handle, len(r), rp, out.ctypes.data_as(C.POINTER(C.c_double))))
    return out[0::2] + 1j * out[1::2]


def get_links(lat: Lattice) -> np.ndarray:
    out = np.empty((lat.T, lat.L, lat.L, lat.L, 4))
    _check(load_library().u1ml_get_links(lat.handle, out.ctypes.data_as(C.POINTER(C.c_double))))
    return out


def set_links(lat: Lattice, th: np.ndarray):
    a = np.ascontiguousarray(th, dtype=np.float64)
    if a.size != 4 * lat.V:
        raise ValueError("wrong number of link angles")
    _check(load_library().u1ml_set_links(lat.handle, a.ctypes.data_as(C.POINTER(C.c_double))))


def get_pass_id(lat: Lattice) -> int:
    v = C.c_uint64()
    _check(load_library().u1ml_get_pass_id(lat.handle, C.byref(v)))
    return int(v.value)


def set_pass_id(lat: Lattice, pass_id: int):
    _check(load_library().u1ml_set_pass_id(lat.handle, int(pass_id)))


MULTIHIT = 1
FIELD_SQUARED = 2
SYMMETRIC = 4


def _estimator_flags(multihit: bool, field_squared: bool, symmetric: bool) -> int:
    return (MULTIHIT if multihit else 0) | (FIELD_SQUARED if field_squared else 0) | (SYMMETRIC if symmetric else 0)


def set_estimator(lat: Lattice, multihit: bool = False, field_squared: bool = False, symmetric: bool = False):
    """Estimator options of the following multilevel runs (u1ml_set_estimator)."""
    _check(load_library().u1ml_set_estimator(lat.handle, _estimator_flags(multihit, field_squared, symmetric)))


def set_debug(lat: Lattice, flags: int, capacity: int = 0):
    _check(load_library().u1ml_set_debug(lat.handle, flags, capacity))


def get_accept_log(lat: Lattice) -> np.ndarray:
    lib = load_library()
    n = C.c_size_t()
    _check(lib.u1ml_get_accept_log(lat.handle, None, 0, C.byref(n)))
    out = np.zeros(n.value, dtype=np.uint8)
    if n.value:
        _check(lib.u1ml_get_accept_log(lat.handle, out.ctypes.data_as(C.POINTER(C.c_uint8)), n.value, C.byref(n)))
    return out


def save(lat: Lattice, path: str):
    _check(load_library().u1ml_save(lat.handle, path.encode()))


def load(lat: Lattice, path: str):
    _check(load_library().u1ml_load(lat.handle, path.encode()))


def synchronize(lat: Lattice):
    _check(load_library().u1ml_synchronize(lat.handle))


def autotune(lat: Lattice) -> int:
    b = C.c_int()
    _check(load_library().u1ml_autotune(lat.handle, C.byref(b)))
    return int(b.value)


def get_tuning(obj) -> dict:
    """Launch shapes of a Lattice or Batch (u1ml_get_tuning / u1ml_batch_get_tuning)."""
    t = Tuning()
    lib = load_library()
    f = lib.u1ml_batch_get_tuning if isinstance(obj, Batch) else lib.u1ml_get_tuning
    _check(f(obj.handle, C.byref(t)))
    return t.as_dict()


def set_tuning(obj, **values):
    """Change some launch shapes of a Lattice or Batch; the others keep their values."""
    cur = get_tuning(obj)
    unknown = set(values) - set(cur)
    if unknown:
        raise U1MLError(EINVAL, f"unknown tuning fields {sorted(unknown)}")
    cur.update(values)
    t = Tuning(**cur)
    lib = load_library()
    f = lib.u1ml_batch_set_tuning if isinstance(obj, Batch) else lib.u1ml_set_tuning
    _check(f(obj.handle, C.byref(t)))


def batch_autotune(b, slab_sizes=(), n_sub=(), r_list=(), rf_list=()) -> dict:
    """u1ml_batch_autotune; with slab_sizes empty only the class passes are tuned."""
    th, thp = _ints(slab_sizes if len(slab_sizes) else [0])
    ns, nsp = _ints(n_sub if len(n_sub) else [0])
    r, rp = _ints(r_list if len(r_list) else [0])
    rf, rfp = _ints(rf_list if len(rf_list) else [0])
    t = Tuning()
    _check(load_library().u1ml_batch_autotune(b.handle, len(slab_sizes), thp if len(slab_sizes) else None,
                                              nsp if len(slab_sizes) else None, len(r_list),
                                              rp if len(r_list) else None, len(rf_list),
                                              rfp if len(rf_list) else None, C.byref(t)))
    return t.as_dict()


def stream_bandwidth(kind: str, n_bytes: int, reps: int = 5) -> float:
    """u1ml_stream_bandwidth: GB/s of a plain read ("read") or copy ("copy") stream."""
    out = C.c_double()
    _check(load_library().u1ml_stream_bandwidth({"read": 0, "copy": 1}[kind], int(n_bytes), int(reps),
                                                C.byref(out)))
    return float(out.value)


def profile_sweeps(lat: Lattice, n_sweeps: int, n_metro: int = 1, n_or: int = 3):
    """Average class-pass kernel durations in microseconds: (Metropolis, OR)."""
    out = np.zeros(2)
    _check(load_library().u1ml_profile_sweeps(lat.handle, n_sweeps, n_metro, n_or,
                                              out.ctypes.data_as(C.POINTER(C.c_double))))
    return float(out[0]), float(out[1])


def batch_profile_sweeps(b, n_sweeps: int, n_metro: int = 1, n_or: int = 3):
    """Average class-pass kernel durations in microseconds for a batch: (Metropolis, OR)."""
    out = np.zeros(2)
    _check(load_library().u1ml_batch_profile_sweeps(b.handle, n_sweeps, n_metro, n_or,
                                                    out.ctypes.data_as(C.POINTER(C.c_double))))
    return float(out[0]), float(out[1])


class Batch:
    """Many lattices updated by the same launches: wraps a ``u1ml_batch*``."""

    def __init__(self, handle, L, T, beta, seed):
        self._h = handle
        self.L, self.T, self.beta, self.seed = list(L), list(T), list(beta), list(seed)
        self._n_r = None  # None: r = 1..T/2 of the last cycle
        self._n_rf = 0
        self._destroy = load_library().u1ml_batch_destroy

    def __del__(self):
        self.close()

    def close(self):
        if getattr(self, "_h", None):
            self._destroy(self._h)
            self._h = None

    @property
    def handle(self):
        return self._h


def batch_create(L, T, beta, seed, *, start: int = HOT, precision: int = FP64, eps: float = 1.0,
                 block: int = 0, stream=None, graphs: bool = True) -> Batch:
    lib = load_library()
    n = len(L)
    o = default_options()
    o.start, o.precision, o.eps, o.block = start, precision, float(eps), block
    o.no_graphs = 0 if graphs else 1
    if stream is not None:
        o.stream = C.c_void_p(int(stream))
    La, Lp = _ints(L)
    Ta, Tp = _ints(T)
    b = np.ascontiguousarray(beta, dtype=np.float64)
    s = np.ascontiguousarray(seed, dtype=np.uint64)
    h = C.c_void_p()
    _check(lib.u1ml_batch_create(n, Lp, Tp, b.ctypes.data_as(C.POINTER(C.c_double)),
                                 s.ctypes.data_as(C.POINTER(C.c_uint64)), C.byref(o), C.byref(h)))
    return Batch(h, L, T, beta, seed)


def batch_sweep(b: Batch, n_metro: int = 1, n_or: int = 3):
    _check(load_library().u1ml_batch_sweep(b.handle, n_metro, n_or))


def batch_cycle(b: Batch, n_sweeps: int, n_metro: int, n_or: int, th: int, n_sub: int, use_graph: bool = True):
    _check(load_library().u1ml_batch_cycle(b.handle, n_sweeps, n_metro, n_or, th, n_sub, int(bool(use_graph))))
    b._n_r, b._n_rf = None, 0


def batch_multilevel(b: Batch, slab_sizes, n_sub, n_metro: int = 1, n_or: int = 3, r_list=(1,), rf_list=()):
    th, thp = _ints(slab_sizes)
    ns, nsp = _ints(n_sub)
    r, rp = _ints(r_list)
    rf, rfp = _ints(rf_list if len(rf_list) else [0])
    _check(load_library().u1ml_batch_multilevel(b.handle, len(th), thp, nsp, n_metro, n_or, len(r), rp,
                                                len(rf_list), rfp if len(rf_list) else None))
    b._n_r, b._n_rf = [len(r)] * len(b.L), len(rf_list)


def batch_set_estimator(b: Batch, multihit: bool = False, field_squared: bool = False, symmetric: bool = False):
    _check(load_library().u1ml_batch_set_estimator(b.handle, _estimator_flags(multihit, field_squared, symmetric)))


def batch_ensemble_reset(b: Batch):
    _check(load_library().u1ml_batch_ensemble_reset(b.handle))


def batch_ensemble_add(b: Batch):
    _check(load_library().u1ml_batch_ensemble_add(b.handle))


def batch_ensemble_read(b: Batch, i: int, correlator: bool = True, field_profile: bool = False,
                        connected: bool = False):
    lib = load_library()
    return _ensemble_read(lambda *a: lib.u1ml_batch_ensemble_info(b.handle, i, *a),
                          lambda *a: lib.u1ml_batch_ensemble_read(b.handle, i, *a), b.L[i], correlator,
                          field_profile, connected)


def batch_measure(b: Batch, i: int, correlator: bool = True, field_profile: bool = False):
    """Returns (obs dict, correlator complex[n_r] or None, field complex[n_rf][2][6][L][L] or None)."""
    obs = Observables()
    nr = b._n_r[i] if b._n_r is not None else b.T[i] // 2
    corr = np.zeros(2 * nr) if correlator else None
    L = b.L[i]
    fp = np.zeros(b._n_rf * 2 * 6 * L * L * 2) if field_profile else None
    _check(load_library().u1ml_batch_measure(
        b.handle, i, C.byref(obs), corr.ctypes.data_as(C.POINTER(C.c_double)) if correlator else None,
        fp.ctypes.data_as(C.POINTER(C.c_double)) if field_profile else None))
    f = None
    if fp is not None:
        f = fp.reshape(b._n_rf, 2, 6, L, L, 2)
        f = f[..., 0] + 1j * f[..., 1]
    return obs.as_dict(), (corr[0::2] + 1j * corr[1::2]) if correlator else None, f


def batch_get_links(b: Batch, i: int) -> np.ndarray:
    out = np.empty((b.T[i], b.L[i], b.L[i], b.L[i], 4))
    _check(load_library().u1ml_batch_get_links(b.handle, i, out.ctypes.data_as(C.POINTER(C.c_double))))
    return out


def batch_set_links(b: Batch, i: int, th: np.ndarray):
    a = np.ascontiguousarray(th, dtype=np.float64)
    _check(load_library().u1ml_batch_set_links(b.handle, i, a.ctypes.data_as(C.POINTER(C.c_double))))


def batch_get_pass_id(b: Batch, i: int) -> int:
    v = C.c_uint64()
    _check(load_library().u1ml_batch_get_pass_id(b.handle, i, C.byref(v)))
    return int(v.value)


def batch_set_pass_id(b: Batch, i: int, pass_id: int):
    _check(load_library().u1ml_batch_set_pass_id(b.handle, i, int(pass_id)))


def batch_save(b: Batch, path: str):
    _check(load_library().u1ml_batch_save(b.handle, path.encode()))


def batch_load(b: Batch, path: str):
    _check(load_library().u1ml_batch_load(b.handle, path.encode()))


def batch_synchronize(b: Batch):
    _check(load_library().u1ml_batch_synchronize(b.handle))
