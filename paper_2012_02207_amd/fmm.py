"""Python binding of the gfx950 FMM library (``libfmm_hip.so``, C ABI in include/fmm.h).

Argument marshalling only: every stage of the force pass runs in the HIP
kernels behind the C ABI.  PyTorch supplies device memory and the current HIP
stream.  There is no CPU fallback: if the library cannot be loaded, or no GPU
is present, every entry point raises.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfmm_hip.so")

FMM_OK, FMM_EINVAL, FMM_ENOMEM, FMM_EHIP, FMM_ENOTBUILT, FMM_EDATA, FMM_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
PRECISION = {"fp64": 0, "mixed": 1, "direct": 2}
MAC = {"error": 0, "geometric": 1}
EXPORTS = dict(keys=(0, np.uint64), perm=(1, np.int32), cell_level=(2, np.int32),
               cell_begin=(3, np.int32), cell_end=(4, np.int32), cell_parent=(5, np.int32),
               cell_child0=(6, np.int32), cell_nchild=(7, np.int32), cell_mass=(8, np.float64),
               cell_com=(9, np.float64), cell_rad=(10, np.float64), mult=(11, np.float64),
               pk=(12, np.float64), fcell_est=(13, np.float64), f_part=(14, np.float64),
               fmin=(15, np.float64), est_far=(16, np.int32), est_near=(17, np.int32),
               m2l=(18, np.int32), p2p=(19, np.int32), local=(20, np.float64),
               rootbox=(21, np.float64))
SYMBOLS = ["fmm_default_params", "fmm_create", "fmm_set_params", "fmm_get_params", "fmm_build", "fmm_forces",
           "fmm_forces_noalloc", "fmm_forces_batch", "fmm_forces_frozen",
           "fmm_forces_frozen_graph", "fmm_autotune", "fmm_adjoint", "fmm_adjoint_last",
           "fmm_jerk", "fmm_stats", "fmm_export", "fmm_set_workspace_limit",
           "fmm_direct", "fmm_strerror", "fmm_last_error", "fmm_destroy"]


NOALLOC_MAX_N = 65536  # FMM_NOALLOC_MAX_N of include/fmm.h


class FmmError(RuntimeError):
    def __init__(self, status, msg=""):
        self.status = status
        super().__init__(f"{_strerror(status)} ({status}){': ' + msg if msg else ''}")


class Params(C.Structure):
    _fields_ = [("p", C.c_int), ("err_tol", C.c_double), ("theta", C.c_double),
                ("theta_est", C.c_double), ("n_leaf", C.c_int), ("precision", C.c_int),
                ("mac", C.c_int), ("check_inputs", C.c_int), ("root_levels", C.c_int),
                ("m2l_waves", C.c_int), ("p2p_groups", C.c_int),
                ("p2p_start", C.c_int)]


class Stats(C.Structure):
    _fields_ = [("n", C.c_int64), ("ncell", C.c_int64), ("nleaf", C.c_int64), ("depth", C.c_int32),
                ("n_m2l", C.c_int64), ("n_p2p_cells", C.c_int64), ("n_p2p_pairs", C.c_int64),
                ("n_est_far", C.c_int64), ("n_est_near", C.c_int64), ("n_m2l_fp32", C.c_int64),
                ("ms_tree", C.c_double), ("ms_upward", C.c_double), ("ms_estimate", C.c_double),
                ("ms_walk", C.c_double), ("ms_m2l", C.c_double), ("ms_local", C.c_double),
                ("ms_p2p", C.c_double), ("ms_total", C.c_double), ("workspace_bytes", C.c_size_t),
                ("nsys", C.c_int64), ("ms_m2l_kernel", C.c_double), ("ms_sort", C.c_double),
                ("ms_gather", C.c_double), ("ms_walk_steps", C.c_double), ("n_p2p_items", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load_library():
    """Loads libfmm_hip.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2012_02207_amd.build.build()")
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    lib.fmm_default_params.argtypes = [C.POINTER(Params)]
    lib.fmm_create.argtypes = [C.POINTER(C.c_void_p), C.POINTER(Params)]
    lib.fmm_set_params.argtypes = [P, C.POINTER(Params)]
    lib.fmm_get_params.argtypes = [P, C.POINTER(Params)]
    lib.fmm_build.argtypes = [P, C.c_int64, P, P, P]
    lib.fmm_forces.argtypes = [P, C.c_int64, P, P, C.c_double, C.c_int, C.c_double, P, P, P]
    lib.fmm_forces_noalloc.argtypes = [P, C.c_int64, P, P, C.c_double, C.c_int, C.c_double, P, P, P]
    lib.fmm_forces_batch.argtypes = [P, C.c_int64, C.POINTER(C.c_int64), P, P, C.c_double, C.c_int,
                                     C.c_double, P, P, P]
    lib.fmm_autotune.argtypes = [P, C.c_int64, C.POINTER(C.c_int64), P, P, C.c_double, C.c_int,
                                 C.c_double, P, P, P, C.POINTER(C.c_int)]
    lib.fmm_jerk.argtypes = [P, C.c_int64, P, P, P, C.c_double, C.c_int, C.c_double, P, P, P, P]
    lib.fmm_forces_frozen.argtypes = [P, C.c_int64, P, P, C.c_double, P, P, P]
    lib.fmm_forces_frozen_graph.argtypes = [P, C.c_int64, P, P, C.c_double, P, P, P]
    lib.fmm_adjoint.argtypes = [P, C.c_int64, P, P, C.c_double, C.c_int, C.c_double, P, P, P, P, P]
    lib.fmm_adjoint_last.argtypes = [P, C.c_int64, P, P, P, P, P, P]
    lib.fmm_stats.argtypes = [P, C.POINTER(Stats)]
    lib.fmm_export.argtypes = [P, C.c_int, P, C.c_size_t]
    lib.fmm_set_workspace_limit.argtypes = [P, C.c_size_t]
    lib.fmm_direct.argtypes = [C.c_int64, P, P, C.c_double, C.c_int64, P, P, P, P]
    lib.fmm_strerror.argtypes = [C.c_int]
    lib.fmm_strerror.restype = C.c_char_p
    lib.fmm_last_error.argtypes = [P]
    lib.fmm_last_error.restype = C.c_char_p
    lib.fmm_destroy.argtypes = [P]
    for f in ("fmm_create", "fmm_set_params", "fmm_get_params", "fmm_build", "fmm_forces", "fmm_forces_noalloc", "fmm_forces_batch",
              "fmm_forces_frozen", "fmm_forces_frozen_graph", "fmm_autotune", "fmm_adjoint", "fmm_adjoint_last", "fmm_jerk", "fmm_stats", "fmm_export",
              "fmm_set_workspace_limit", "fmm_direct"):
        getattr(lib, f).restype = C.c_int
    _lib = lib
    return lib


def _strerror(status):
    try:
        return load_library().fmm_strerror(status).decode()
    except ImportError:
        return f"status {status}"


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the FMM library needs a ROCm GPU; none is visible")
    return torch


def _dev_ptr(t, dtype, shape, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return C.c_void_p(t.data_ptr())


def _stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def default_params():
    p = Params()
    load_library().fmm_default_params(C.byref(p))
    return p


class FMM:
    """A force-evaluation context (owns the device workspace)."""

    def __init__(self, p=10, err_tol=1e-7, theta=1.0, theta_est=1.0, n_leaf=64, precision="fp64",
                 mac="error", check_inputs=False, root_levels=3, m2l_waves=1, p2p_groups=0,
                 p2p_start=0):
        lib = load_library()
        _torch()
        self._lib = lib
        self.params = default_params()
        self.params.p, self.params.err_tol, self.params.theta = int(p), float(err_tol), float(theta)
        self.params.theta_est, self.params.n_leaf = float(theta_est), int(n_leaf)
        self.params.precision, self.params.mac = PRECISION[precision], MAC[mac]
        self.params.check_inputs, self.params.root_levels = int(bool(check_inputs)), int(root_levels)
        self.params.m2l_waves, self.params.p2p_groups = int(m2l_waves), int(p2p_groups)
        self.params.p2p_start = int(p2p_start)
        h = C.c_void_p()
        st = lib.fmm_create(C.byref(h), C.byref(self.params))
        if st != FMM_OK:
            raise FmmError(st)
        self._h = h
        self.n = 0
        # calls that changed the context's tree and expansions; fmm_adjoint_last
        # needs the state of the latest one
        self.evals = 0

    def close(self):
        if getattr(self, "_h", None):
            self._lib.fmm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != FMM_OK:
            raise FmmError(st, self._lib.fmm_last_error(self._h).decode())

    def set_params(self, **kw):
        """Replaces parameters for later calls (fmm_set_params): any of p, err_tol,
        theta, theta_est, n_leaf, precision ("fp64"/"mixed"/"direct"), mac,
        check_inputs, root_levels, m2l_waves, p2p_groups, p2p_start."""
        conv = {"precision": lambda v: PRECISION[v], "mac": lambda v: MAC[v],
                "check_inputs": lambda v: int(bool(v))}
        new = Params()
        C.pointer(new)[0] = self.params
        for k, v in kw.items():
            if not hasattr(new, k):
                raise ValueError(f"unknown parameter {k}")
            setattr(new, k, conv.get(k, lambda x: x)(v))
        self._check(self._lib.fmm_set_params(self._h, C.byref(new)))
        self.params = new

    def set_workspace_limit(self, nbytes):
        self._check(self._lib.fmm_set_workspace_limit(self._h, int(nbytes)))

    def build(self, pos, mass):
        torch = _torch()
        n = mass.shape[0]
        self._check(self._lib.fmm_build(self._h, n, _dev_ptr(pos, torch.float64, (n, 3), "pos"),
                                        _dev_ptr(mass, torch.float64, (n,), "mass"), _stream()))
        self.n = n
        self.evals += 1

    def forces(self, pos, mass, eps_soft=0.0, p=None, err_tol=None, out=None, noalloc=False):
        """acc (n, 3) and pot (n,) as new (or given) float64 device tensors.
        noalloc=True calls fmm_forces_noalloc (scratch in the library's static
        device array; n <= NOALLOC_MAX_N)."""
        torch = _torch()
        n = mass.shape[0]
        pp = _dev_ptr(pos, torch.float64, (n, 3), "pos")
        mp = _dev_ptr(mass, torch.float64, (n,), "mass")
        if out is None:
            acc = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
            pot = torch.empty((n,), dtype=torch.float64, device=pos.device)
        else:
            acc, pot = out
        fn = self._lib.fmm_forces_noalloc if noalloc else self._lib.fmm_forces
        self._check(fn(
            self._h, n, pp, mp, float(eps_soft), int(self.params.p if p is None else p),
            float(self.params.err_tol if err_tol is None else err_tol),
            _dev_ptr(acc, torch.float64, (n, 3), "acc"), _dev_ptr(pot, torch.float64, (n,), "pot"),
            _stream()))
        if not noalloc:  # the allocation-free call leaves the context's exports alone
            self.n = n
            self.evals += 1
            self.last_p = int(self.params.p if p is None else p)
        return acc, pot

    def forces_batch(self, pos, mass, offsets, eps_soft=0.0, p=None, err_tol=None, out=None):
        """Independent systems in one pass: system s is bodies offsets[s]:offsets[s+1]
        (host integers, offsets[0] = 0, strictly increasing).  Returns acc, pot."""
        torch = _torch()
        n = mass.shape[0]
        off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        if off.ndim != 1 or off.size < 2 or off[-1] != n:
            raise ValueError("offsets must be a 1-D host array ending at the body count")
        pp = _dev_ptr(pos, torch.float64, (n, 3), "pos")
        mp = _dev_ptr(mass, torch.float64, (n,), "mass")
        if out is None:
            acc = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
            pot = torch.empty((n,), dtype=torch.float64, device=pos.device)
        else:
            acc, pot = out
        self._check(self._lib.fmm_forces_batch(
            self._h, off.size - 1, off.ctypes.data_as(C.POINTER(C.c_int64)), pp, mp, float(eps_soft),
            int(self.params.p if p is None else p),
            float(self.params.err_tol if err_tol is None else err_tol),
            _dev_ptr(acc, torch.float64, (n, 3), "acc"), _dev_ptr(pot, torch.float64, (n,), "pot"),
            _stream()))
        self.n = n
        self.evals += 1
        self.last_p = int(self.params.p if p is None else p)
        return acc, pot

    def autotune(self, pos, mass, offsets=None, eps_soft=0.0, p=None, err_tol=None):
        """Picks n_leaf, then (mixed precision) the FP32 M2L's wavefronts per
        sink, then the near field's lane groups for this workload (timed on the
        GPU, cached per workload class in the process); returns n_leaf.  All
        choices are set in the context and read back into self.params."""
        torch = _torch()
        n = mass.shape[0]
        off = np.ascontiguousarray(np.asarray([0, n] if offsets is None else offsets, dtype=np.int64))
        acc = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
        pot = torch.empty((n,), dtype=torch.float64, device=pos.device)
        chosen = C.c_int(0)
        self._check(self._lib.fmm_autotune(
            self._h, off.size - 1, off.ctypes.data_as(C.POINTER(C.c_int64)),
            _dev_ptr(pos, torch.float64, (n, 3), "pos"), _dev_ptr(mass, torch.float64, (n,), "mass"),
            float(eps_soft), int(self.params.p if p is None else p),
            float(self.params.err_tol if err_tol is None else err_tol),
            _dev_ptr(acc, torch.float64, (n, 3), "acc"), _dev_ptr(pot, torch.float64, (n,), "pot"),
            _stream(), C.byref(chosen)))
        self.evals += 1
        self.params = self.get_params()
        return chosen.value

    def get_params(self):
        """The context's current parameters (fmm_get_params), as a Params struct."""
        out = Params()
        self._check(self._lib.fmm_get_params(self._h, C.byref(out)))
        return out

    def forces_frozen(self, pos, mass, eps_soft=0.0, out=None, graph=False):
        """Forces with the tree and lists of the last evaluation kept (see fmm_forces_frozen);
        graph=True replays the evaluation as a captured HIP graph (fmm_forces_frozen_graph)."""
        torch = _torch()
        n = mass.shape[0]
        if out is None:
            acc = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
            pot = torch.empty((n,), dtype=torch.float64, device=pos.device)
        else:
            acc, pot = out
        fn = self._lib.fmm_forces_frozen_graph if graph else self._lib.fmm_forces_frozen
        self._check(fn(
            self._h, n, _dev_ptr(pos, torch.float64, (n, 3), "pos"),
            _dev_ptr(mass, torch.float64, (n,), "mass"), float(eps_soft),
            _dev_ptr(acc, torch.float64, (n, 3), "acc"), _dev_ptr(pot, torch.float64, (n,), "pot"),
            _stream()))
        self.evals += 1
        return acc, pot

    def jerk(self, pos, vel, mass, eps_soft=0.0, p=None, err_tol=None):
        """(acc, pot, jerk): forces and their time derivative along the motion."""
        torch = _torch()
        n = mass.shape[0]
        acc = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
        pot = torch.empty((n,), dtype=torch.float64, device=pos.device)
        jerk = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
        self._check(self._lib.fmm_jerk(
            self._h, n, _dev_ptr(pos, torch.float64, (n, 3), "pos"),
            _dev_ptr(vel, torch.float64, (n, 3), "vel"), _dev_ptr(mass, torch.float64, (n,), "mass"),
            float(eps_soft), int(self.params.p if p is None else p),
            float(self.params.err_tol if err_tol is None else err_tol),
            _dev_ptr(acc, torch.float64, (n, 3), "acc"), _dev_ptr(pot, torch.float64, (n,), "pot"),
            _dev_ptr(jerk, torch.float64, (n, 3), "jerk"), _stream()))
        self.n = n
        self.evals += 1
        return acc, pot, jerk

    def adjoint(self, pos, mass, gacc, gpot=None, eps_soft=0.0, p=None, err_tol=None):
        """(dL/dpos, dL/dmass) for dL/dacc = gacc and dL/dpot = gpot (or zero);
        recomputes the forward pass at pos."""
        torch = _torch()
        n = mass.shape[0]
        gpos = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
        gmass = torch.empty((n,), dtype=torch.float64, device=pos.device)
        gp = None if gpot is None else _dev_ptr(gpot, torch.float64, (n,), "gpot")
        self._check(self._lib.fmm_adjoint(
            self._h, n, _dev_ptr(pos, torch.float64, (n, 3), "pos"),
            _dev_ptr(mass, torch.float64, (n,), "mass"), float(eps_soft),
            int(self.params.p if p is None else p),
            float(self.params.err_tol if err_tol is None else err_tol),
            _dev_ptr(gacc, torch.float64, (n, 3), "gacc"), gp,
            _dev_ptr(gpos, torch.float64, (n, 3), "gpos"), _dev_ptr(gmass, torch.float64, (n,), "gmass"),
            _stream()))
        self.n = n
        self.evals += 1
        return gpos, gmass

    def adjoint_last(self, acc, gacc, gpot=None):
        """(dL/dpos, dL/dmass) at the positions and masses of this context's last
        evaluation (one FP64 system; acc is the acceleration it returned), reusing
        its tree, lists and expansions (fmm_adjoint_last): fmm_adjoint's result
        without its forward pass."""
        torch = _torch()
        n = acc.shape[0]
        gpos = torch.empty((n, 3), dtype=torch.float64, device=acc.device)
        gmass = torch.empty((n,), dtype=torch.float64, device=acc.device)
        gp = None if gpot is None else _dev_ptr(gpot, torch.float64, (n,), "gpot")
        self._check(self._lib.fmm_adjoint_last(
            self._h, n, _dev_ptr(acc, torch.float64, (n, 3), "acc"),
            _dev_ptr(gacc, torch.float64, (n, 3), "gacc"), gp,
            _dev_ptr(gpos, torch.float64, (n, 3), "gpos"), _dev_ptr(gmass, torch.float64, (n,), "gmass"),
            _stream()))
        return gpos, gmass

    def stats(self):
        s = Stats()
        self._check(self._lib.fmm_stats(self._h, C.byref(s)))
        return s.as_dict()

    def export(self, name):
        what, dt = EXPORTS[name]
        st = self.stats()
        nc, n = st["ncell"], st["n"]
        p = getattr(self, "last_p", self.params.p)
        k = (p + 1) * (p + 2) // 2
        count = {"keys": n, "perm": n, "f_part": n, "cell_com": 3 * nc, "mult": nc * k * 2,
                 "local": nc * k * 2, "pk": nc * (p + 1), "rootbox": 5 * st["nsys"],
                 "est_far": 2 * st["n_est_far"], "est_near": 2 * st["n_est_near"],
                 "m2l": 2 * st["n_m2l"], "p2p": 2 * st["n_p2p_cells"]}.get(name, nc)
        buf = np.empty(max(int(count), 1), dtype=dt)
        self._check(self._lib.fmm_export(self._h, what, buf.ctypes.data_as(C.c_void_p), buf.nbytes))
        buf = buf[:count]
        if name in ("est_far", "est_near", "m2l", "p2p"):
            return buf.reshape(-1, 2)
        if name == "cell_com":
            return buf.reshape(nc, 3)
        if name in ("mult", "local"):
            b = buf.reshape(nc, k, 2)
            return b[..., 0] + 1j * b[..., 1]
        if name == "pk":
            return buf.reshape(nc, p + 1)
        return buf


def forces(pos, mass, eps_soft=0.0, p=10, err_tol=1e-7, precision="fp64", n_leaf=64, **kw):
    """One force evaluation with a temporary context: returns (acc, pot)."""
    f = FMM(p=p, err_tol=err_tol, precision=precision, n_leaf=n_leaf, **kw)
    try:
        return f.forces(pos, mass, eps_soft=eps_soft)
    finally:
        f.close()


def direct(pos, mass, eps_soft=0.0, sinks=None):
    """O(N^2) direct sum on the GPU for the given sinks (int32 device tensor) or all."""
    torch = _torch()
    lib = load_library()
    n = mass.shape[0]
    ns = n if sinks is None else sinks.shape[0]
    acc = torch.empty((ns, 3), dtype=torch.float64, device=pos.device)
    pot = torch.empty((ns,), dtype=torch.float64, device=pos.device)
    sp = None if sinks is None else _dev_ptr(sinks, torch.int32, (ns,), "sinks")
    st = lib.fmm_direct(n, _dev_ptr(pos, torch.float64, (n, 3), "pos"),
                        _dev_ptr(mass, torch.float64, (n,), "mass"), float(eps_soft), ns, sp,
                        _dev_ptr(acc, torch.float64, (ns, 3), "acc"),
                        _dev_ptr(pot, torch.float64, (ns,), "pot"), _stream())
    if st != FMM_OK:
        raise FmmError(st)
    return acc, pot
