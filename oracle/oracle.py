"""ctypes binding of the C oracle (``oracle/fmm_oracle.c``) -- test infrastructure only.

The oracle is a plain FP64 CPU restatement of the paper's force pass
(section 2) and of the direct sum it approximates; see the C sources for the
section-by-section citations.
"""
import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
          "-std=c99", "-Wall", "-Wno-unused-function"]


def lib_path():
    return _SO


def build(force=True):
    """Compile the oracle with gcc (no contraction, no fast-math)."""
    if not force and os.path.exists(_SO):
        return _SO
    src = os.path.join(_HERE, "fmm_oracle.c")
    tmp = _SO + ".tmp"
    subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, src, "-lm"])
    os.replace(tmp, _SO)
    return _SO


_lib = None


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = C.CDLL(_SO)
        P = C.c_void_p
        lib.orc_new.restype = P
        lib.orc_free.argtypes = [P]
        lib.orc_run.argtypes = [P, C.c_int64, P, P, C.c_double, C.c_int, C.c_double, C.c_double,
                                C.c_double, C.c_int, C.c_int, C.c_int, C.c_int, P, P, P]
        lib.orc_run.restype = C.c_int
        lib.orc_get.argtypes = [P, C.c_int, C.POINTER(C.c_void_p)]
        lib.orc_get.restype = C.c_int64
        lib.orc_ncell.argtypes = [P]
        lib.orc_ncell.restype = C.c_int64
        lib.orc_direct.argtypes = [C.c_int64, P, P, C.c_double, C.c_int64, P, C.c_int, P, P]
        lib.orc_direct.restype = C.c_int
        for f in ("orc_regular", "orc_irregular"):
            getattr(lib, f).argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, P, P]
        for f in ("orc_m2l_direct", "orc_m2l_rotated", "orc_l2l", "orc_m2m"):
            getattr(lib, f).argtypes = [C.c_int, P, P, P, P, P]
        lib.orc_l2p.argtypes = [C.c_int, P, P, P, P, P]
        lib.orc_p2m.argtypes = [C.c_int, C.c_int64, P, P, P, P, P]
        lib.orc_pk.argtypes = [C.c_int, P, P, P]
        lib.orc_swap_table.argtypes = [C.c_int]
        lib.orc_swap_table.restype = C.POINTER(C.c_double)
        lib.orc_factorials.restype = C.POINTER(C.c_double)
        lib.orc_threads.restype = C.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def ncoef(p):
    return (p + 1) * (p + 2) // 2


STAGES = {"tree": 1, "upward": 2, "estimate": 3, "walk": 4, "eval": 5}
_GET = dict(keys=(0, np.uint64), perm=(1, np.int64), cell_level=(2, np.int32),
            cell_begin=(3, np.int64), cell_end=(4, np.int64), cell_parent=(5, np.int64),
            cell_child0=(6, np.int64), cell_nchild=(7, np.int32), cell_mass=(8, np.float64),
            cell_com=(9, np.float64), cell_rad=(10, np.float64), mult=(11, np.float64),
            pk=(12, np.float64), fcell_est=(13, np.float64), f_part=(14, np.float64),
            fmin=(15, np.float64), est_far=(16, np.int64), est_near=(17, np.int64),
            m2l=(18, np.int64), p2p=(19, np.int64), local=(20, np.float64),
            rootbox=(21, np.float64), sorted_pos=(22, np.float64))


class Oracle:
    """One oracle force pass; exported arrays are copied into numpy on demand."""

    def __init__(self):
        self._c = _L().orc_new()
        self.p = None

    def __del__(self):
        if getattr(self, "_c", None):
            _L().orc_free(self._c)
            self._c = None

    def run(self, pos, mass, eps_soft=0.0, p=6, err_tol=1e-6, theta=1.0, theta_est=1.0,
            n_leaf=64, mac="error", m2l="rotation", stage="eval", eval_mask=None):
        pos = np.ascontiguousarray(pos, dtype=np.float64)
        mass = np.ascontiguousarray(mass, dtype=np.float64)
        n = mass.shape[0]
        assert pos.shape == (n, 3)
        st = STAGES[stage]
        acc = np.empty((n, 3)) if st == 5 else None
        pot = np.empty(n) if st == 5 else None
        mask = None
        if eval_mask is not None:
            mask = np.ascontiguousarray(eval_mask, dtype=np.uint8)
            assert mask.shape == (n,)
        rc = _L().orc_run(self._c, n, _ptr(pos), _ptr(mass), float(eps_soft), int(p),
                          float(err_tol), float(theta), float(theta_est), int(n_leaf),
                          0 if mac == "error" else 1, 0 if m2l == "rotation" else 1, st,
                          _ptr(mask), _ptr(acc), _ptr(pot))
        if rc != 0:
            raise ValueError(f"oracle rejected arguments (rc={rc})")
        self.p = p
        self.n = n
        return acc, pot

    def get(self, name):
        what, dt = _GET[name]
        ptr = C.c_void_p()
        cnt = _L().orc_get(self._c, what, C.byref(ptr))
        if cnt == 0 or not ptr.value:
            return np.empty(0, dtype=dt)
        buf = (C.c_char * (cnt * np.dtype(dt).itemsize)).from_address(ptr.value)
        a = np.frombuffer(buf, dtype=dt).copy()
        nc = self.ncell
        if name in ("est_far", "est_near", "m2l", "p2p"):
            a = a.reshape(-1, 2)
        elif name == "cell_com":
            a = a.reshape(nc, 3)
        elif name == "sorted_pos":
            a = a.reshape(-1, 3)
        elif name in ("mult", "local"):
            k = ncoef(self.p)
            a = a.reshape(nc, 2, k)
            a = a[:, 0, :] + 1j * a[:, 1, :]
        elif name == "pk":
            a = a.reshape(nc, self.p + 1)
        return a

    @property
    def ncell(self):
        return int(_L().orc_ncell(self._c))


def direct(pos, mass, eps_soft=0.0, sinks=None, compensated=True):
    """O(N^2) direct sum for the given sinks (all when None), all sources."""
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    mass = np.ascontiguousarray(mass, dtype=np.float64)
    n = mass.shape[0]
    s = None if sinks is None else np.ascontiguousarray(sinks, dtype=np.int64)
    ns = n if s is None else s.shape[0]
    acc = np.empty((ns, 3))
    pot = np.empty(ns)
    rc = _L().orc_direct(n, _ptr(pos), _ptr(mass), float(eps_soft), ns, _ptr(s),
                         1 if compensated else 0, _ptr(acc), _ptr(pot))
    if rc != 0:
        raise ValueError("oracle direct rejected arguments")
    return acc, pot


def _harm(fn, p, x):
    k = ncoef(p)
    re = np.empty(k)
    im = np.empty(k)
    getattr(_L(), fn)(int(p), float(x[0]), float(x[1]), float(x[2]), _ptr(re), _ptr(im))
    return re + 1j * im


def regular(p, x):
    return _harm("orc_regular", p, x)


def irregular(p, x):
    return _harm("orc_irregular", p, x)


def _op(fn, p, coef, vec):
    k = ncoef(p)
    re = np.ascontiguousarray(coef.real, dtype=np.float64)
    im = np.ascontiguousarray(coef.imag, dtype=np.float64)
    v = np.ascontiguousarray(vec, dtype=np.float64)
    ore = np.empty(k)
    oim = np.empty(k)
    getattr(_L(), fn)(int(p), _ptr(re), _ptr(im), _ptr(v), _ptr(ore), _ptr(oim))
    return ore + 1j * oim


def m2l_direct(p, M, R):
    return _op("orc_m2l_direct", p, M, R)


def m2l_rotated(p, M, R):
    return _op("orc_m2l_rotated", p, M, R)


def m2m(p, M, d):
    return _op("orc_m2m", p, M, d)


def l2l(p, Lc, d):
    return _op("orc_l2l", p, Lc, d)


def l2p(p, Lc, X):
    re = np.ascontiguousarray(Lc.real, dtype=np.float64)
    im = np.ascontiguousarray(Lc.imag, dtype=np.float64)
    x = np.ascontiguousarray(X, dtype=np.float64)
    pot = np.empty(1)
    acc = np.empty(3)
    _L().orc_l2p(int(p), _ptr(re), _ptr(im), _ptr(x), _ptr(pot), _ptr(acc))
    return pot[0], acc


def p2m(p, pos, mass, centre):
    """Multipole of the given bodies about `centre` (complex, m >= 0 storage)."""
    pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
    mass = np.ascontiguousarray(mass, dtype=np.float64)
    c = np.ascontiguousarray(centre, dtype=np.float64)
    k = ncoef(p)
    re = np.empty(k)
    im = np.empty(k)
    _L().orc_p2m(int(p), mass.shape[0], _ptr(pos), _ptr(mass), _ptr(c), _ptr(re), _ptr(im))
    return re + 1j * im


def pk(p, M):
    """Per-order norms P_0..P_p of a multipole."""
    re = np.ascontiguousarray(M.real, dtype=np.float64)
    im = np.ascontiguousarray(M.imag, dtype=np.float64)
    out = np.empty(p + 1)
    _L().orc_pk(int(p), _ptr(re), _ptr(im), _ptr(out))
    return out


def swap_table(n):
    d = 2 * n + 1
    ptr = _L().orc_swap_table(int(n))
    return np.ctypeslib.as_array(ptr, shape=(d * d,)).reshape(d, d).copy()


def factorials():
    return np.ctypeslib.as_array(_L().orc_factorials(), shape=(62,)).copy()


def threads():
    return int(_L().orc_threads())
