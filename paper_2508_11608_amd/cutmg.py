"""ctypes binding of libcutmg.so (the C ABI declared in include/cutmg.h).

Argument marshalling only: every step of the multigrid runs in the HIP library.
Vectors are torch tensors on the GPU (float64, contiguous, canonical DoF order
of their level); torch provides the device memory and the current HIP stream.
There is no fallback: without the built library every call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBRARY_PATH = os.path.join(_HERE, "libcutmg.so")

CMG_STATUS = {0: "CMG_OK", -1: "CMG_EINVAL", -2: "CMG_ENOMEM", -3: "CMG_EGEOM", -4: "CMG_ENOTSPD",
              -5: "CMG_ENOTCONV", -6: "CMG_EBREAKDOWN", -7: "CMG_EHIP", 1: "CMG_PENDING"}
CMG_PENDING = 1
CMG_EINVAL = -1


class CutmgError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{CMG_STATUS.get(status, status)}: {message}")
        self.status = status


class LevelSet(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n_shapes", ctypes.c_int),
                ("centers", ctypes.POINTER(ctypes.c_double)), ("semi", ctypes.POINTER(ctypes.c_double)),
                ("box_lo", ctypes.c_double), ("box_hi", ctypes.c_double)]


class Params(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int), ("n_levels", ctypes.c_int), ("coarse_cells", ctypes.c_int),
                ("gamma_D", ctypes.c_double), ("gamma_g", ctypes.c_double), ("ghost_exp_mode", ctypes.c_int),
                ("n_c", ctypes.c_int), ("quad_n", ctypes.c_int), ("precond_fp32", ctypes.c_int),
                ("gamma_m", ctypes.c_double * 3)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("rel_residual", ctypes.c_double), ("n_frac", ctypes.c_double)]


class Request(ctypes.Structure):
    _fields_ = [("levelset", LevelSet), ("params", Params), ("n_modes", ctypes.c_int),
                ("kappa", ctypes.c_void_p), ("amp", ctypes.c_void_p), ("phase", ctypes.c_void_p),
                ("rtol", ctypes.c_double), ("maxit", ctypes.c_int)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("n_dofs", ctypes.c_int64), ("info", SolveInfo), ("cache_hit", ctypes.c_int),
                ("t_submit", ctypes.c_double), ("t_start", ctypes.c_double), ("t_admitted", ctypes.c_double),
                ("t_solve_start", ctypes.c_double), ("t_done", ctypes.c_double), ("batch", ctypes.c_int),
                ("group", ctypes.c_int)]


EXPORTED = ["cmg_setup", "cmg_setup_host", "cmg_set_precision", "cmg_ndofs", "cmg_apply", "cmg_colour_step", "cmg_smooth",
            "cmg_transfer", "cmg_coarse_solve", "cmg_vcycle", "cmg_solve", "cmg_rhs_manufactured", "cmg_rhs_fourier",
            "cmg_export", "cmg_timing", "cmg_timing_read", "cmg_destroy", "cmg_last_error", "cmg_upload",
            "cmg_device_bytes", "cmg_server_create", "cmg_submit", "cmg_poll", "cmg_server_destroy",
            "cmg_vcycle_multi", "cmg_solve_multi", "cmg_gmres", "cmg_vcycle_solve", "cmg_footprint",
            "cmg_set_launch", "cmg_set_ghost_coupling", "cmg_apply_noalloc", "cmg_rhs_fourier_device", "cmg_set_graphs",
            "cmg_group_create", "cmg_group_vcycle", "cmg_group_solve", "cmg_group_destroy"]

_lib = None


def load_library():
    """Load libcutmg.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBRARY_PATH):
        raise RuntimeError(f"{LIBRARY_PATH} is missing: build it with __graft_entry__.build() "
                           "(there is no fallback implementation)")
    lib = ctypes.CDLL(LIBRARY_PATH)
    P, I, D, V = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_void_p
    sig = {
        "cmg_setup": [ctypes.POINTER(LevelSet), ctypes.POINTER(Params), ctypes.POINTER(P)],
        "cmg_setup_host": [ctypes.POINTER(LevelSet), ctypes.POINTER(Params), ctypes.POINTER(P)],
        "cmg_ndofs": [P, I, ctypes.POINTER(ctypes.c_int64)],
        "cmg_set_precision": [P, I],
        "cmg_apply": [P, I, V, V, V],
        "cmg_apply_noalloc": [P, I, V, V, V],
        "cmg_rhs_fourier_device": [P, I, V, V, V, V, V],
        "cmg_colour_step": [P, I, I, I, V, V, V],
        "cmg_smooth": [P, I, I, V, V, V],
        "cmg_transfer": [P, I, I, V, V, V],
        "cmg_coarse_solve": [P, V, V, V],
        "cmg_vcycle": [P, V, V, V],
        "cmg_solve": [P, V, V, D, I, ctypes.POINTER(SolveInfo), V],
        "cmg_vcycle_multi": [P, I, V, V, V],
        "cmg_gmres": [P, V, V, D, I, I, ctypes.POINTER(SolveInfo), V],
        "cmg_vcycle_solve": [P, V, V, D, I, ctypes.POINTER(SolveInfo), V],
        "cmg_solve_multi": [P, I, V, V, D, I, ctypes.POINTER(SolveInfo), V],
        "cmg_rhs_manufactured": [P, ctypes.POINTER(ctypes.c_double)],
        "cmg_rhs_fourier": [P, I, V, V, V, ctypes.POINTER(ctypes.c_double)],
        "cmg_export": [P, I, I, V, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)],
        "cmg_timing": [P, ctypes.c_uint],
        "cmg_upload": [P],
        "cmg_device_bytes": [P, I, ctypes.POINTER(ctypes.c_size_t)],
        "cmg_server_create": [ctypes.c_size_t, I, ctypes.POINTER(P)],
        "cmg_submit": [P, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)],
        "cmg_poll": [P, ctypes.c_uint64, ctypes.POINTER(Result), V, ctypes.c_int64],
        "cmg_timing_read": [P, I, I, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)],
        "cmg_footprint": [ctypes.POINTER(LevelSet), ctypes.POINTER(Params), I, ctypes.POINTER(ctypes.c_size_t),
                          ctypes.POINTER(ctypes.c_int64)],
        "cmg_set_launch": [P, I, I],
        "cmg_set_ghost_coupling": [P, I],
        "cmg_set_graphs": [P, I],
        "cmg_group_create": [ctypes.POINTER(P), I, ctypes.POINTER(P)],
        "cmg_group_vcycle": [P, ctypes.POINTER(V), ctypes.POINTER(V), V],
        "cmg_group_solve": [P, ctypes.POINTER(V), ctypes.POINTER(V), D, I, ctypes.POINTER(SolveInfo),
                            ctypes.POINTER(ctypes.c_int), V],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.cmg_destroy.argtypes = [P]
    lib.cmg_destroy.restype = None
    lib.cmg_server_destroy.argtypes = [P]
    lib.cmg_server_destroy.restype = None
    lib.cmg_group_destroy.argtypes = [P]
    lib.cmg_group_destroy.restype = None
    lib.cmg_last_error.argtypes = []
    lib.cmg_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(status: int):
    if status != 0:
        raise CutmgError(status, _lib.cmg_last_error().decode())


def _dev(t, n=None):
    """Device pointer of a contiguous float64 CUDA tensor (optionally of length n)."""
    import torch

    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError("expected a contiguous float64 tensor on the GPU")
    if n is not None and t.numel() != n:
        raise ValueError(f"expected {n} entries, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    import torch

    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Problem:
    """One CutFEM multigrid hierarchy owned by the library."""

    def __init__(self, workload, device: bool = True, quad_n: int = 14, fp32: bool = False):
        lib = load_library()
        d = workload.dim
        self.workload = workload
        self.dim = d
        self._centers = (ctypes.c_double * (len(workload.centers) * d))(*[v for c in workload.centers for v in c])
        self._semi = (ctypes.c_double * (len(workload.semi) * d))(*[v for s in workload.semi for v in s])
        ls = LevelSet(d, len(workload.centers), self._centers, self._semi, workload.lo, workload.hi)
        prm = _params(workload, quad_n, fp32)
        h = ctypes.c_void_p()
        fn = lib.cmg_setup if device else lib.cmg_setup_host
        _check(fn(ctypes.byref(ls), ctypes.byref(prm), ctypes.byref(h)))
        self._h = h
        self.n_levels = workload.n_levels

    def close(self):
        if getattr(self, "_h", None):
            _lib.cmg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_launch(self, small_cut_launch: int = 1536, max_blocks: int = 2048):
        """Launch shapes by launch size (cmg_set_launch); results are bitwise the same for any choice."""
        _check(_lib.cmg_set_launch(self._h, int(small_cut_launch), int(max_blocks)))

    def set_ghost_coupling(self, patch_local: bool):
        """Cut-patch residuals with the exact ghost coupling (False) or patch-local,
        with x beyond the patch closure taken as zero (True; cmg_set_ghost_coupling)."""
        _check(_lib.cmg_set_ghost_coupling(self._h, int(bool(patch_local))))

    def set_graphs(self, enable: bool):
        """V-cycles as replays of captured HIP graphs (True, default) or kernel by kernel."""
        _check(_lib.cmg_set_graphs(self._h, int(bool(enable))))

    def device_bytes(self, fp32: bool = False, multi: bool = False) -> int:
        n = ctypes.c_size_t()
        _check(_lib.cmg_device_bytes(self._h, int(bool(fp32)) | (2 if multi else 0), ctypes.byref(n)))
        return n.value

    def set_precision(self, fp32: bool):
        """Run the multigrid kernels in FP32 (True) or FP64 (False); CG stays FP64."""
        _check(_lib.cmg_set_precision(self._h, int(bool(fp32))))

    def _lvl(self, level):
        return self.n_levels - 1 if level is None or level < 0 else level

    def ndofs(self, level=None) -> int:
        n = ctypes.c_int64()
        _check(_lib.cmg_ndofs(self._h, self._lvl(level), ctypes.byref(n)))
        return n.value

    def _empty(self, level):
        import torch

        return torch.empty(self.ndofs(level), dtype=torch.float64, device="cuda")

    def apply(self, level, x, y=None):
        level = self._lvl(level)
        y = self._empty(level) if y is None else y
        n = self.ndofs(level)
        _check(_lib.cmg_apply(self._h, level, _dev(x, n), _dev(y, n), _stream()))
        return y

    def apply_noalloc(self, level, x, y):
        """y = A_l x with the library's fixed scratch array (cmg_apply_noalloc);
        y must be given (this call allocates nothing)."""
        level = self._lvl(level)
        n = self.ndofs(level)
        _check(_lib.cmg_apply_noalloc(self._h, level, _dev(x, n), _dev(y, n), _stream()))
        return y

    def colour_step(self, level, interior: bool, colour: int, x, b):
        level = self._lvl(level)
        n = self.ndofs(level)
        _check(_lib.cmg_colour_step(self._h, level, int(bool(interior)), colour, _dev(x, n), _dev(b, n), _stream()))
        return x

    def smooth(self, level, post: bool, x, b):
        level = self._lvl(level)
        n = self.ndofs(level)
        _check(_lib.cmg_smooth(self._h, level, int(bool(post)), _dev(x, n), _dev(b, n), _stream()))
        return x

    def prolongate(self, level, xc, y=None):
        level = self._lvl(level)
        y = self._empty(level) if y is None else y
        _check(_lib.cmg_transfer(self._h, level, 0, _dev(xc, self.ndofs(level - 1)), _dev(y, self.ndofs(level)),
                                 _stream()))
        return y

    def restrict(self, level, xf, y=None):
        level = self._lvl(level)
        y = self._empty(level - 1) if y is None else y
        _check(_lib.cmg_transfer(self._h, level, 1, _dev(xf, self.ndofs(level)), _dev(y, self.ndofs(level - 1)),
                                 _stream()))
        return y

    def coarse_solve(self, b, x=None):
        x = self._empty(0) if x is None else x
        n = self.ndofs(0)
        _check(_lib.cmg_coarse_solve(self._h, _dev(b, n), _dev(x, n), _stream()))
        return x

    def vcycle(self, r, z=None):
        z = self._empty(None) if z is None else z
        n = self.ndofs(None)
        _check(_lib.cmg_vcycle(self._h, _dev(r, n), _dev(z, n), _stream()))
        return z

    def solve(self, b, x=None, rtol=1e-8, maxit=200, raise_on_fail=True):
        x = self._empty(None) if x is None else x
        n = self.ndofs(None)
        info = SolveInfo()
        st = _lib.cmg_solve(self._h, _dev(b, n), _dev(x, n), rtol, maxit, ctypes.byref(info), _stream())
        if raise_on_fail:
            _check(st)
        return x, {"iterations": info.iterations, "rel_residual": info.rel_residual, "n_frac": info.n_frac,
                   "status": st}

    def gmres(self, b, x=None, rtol=1e-9, maxit=500, restart=30, raise_on_fail=True):
        """Right-preconditioned restarted GMRES with the V-cycle (cmg_gmres)."""
        x = self._empty(None) if x is None else x
        n = self.ndofs(None)
        info = SolveInfo()
        st = _lib.cmg_gmres(self._h, _dev(b, n), _dev(x, n), rtol, maxit, restart, ctypes.byref(info), _stream())
        if raise_on_fail:
            _check(st)
        return x, {"iterations": info.iterations, "rel_residual": info.rel_residual, "n_frac": info.n_frac,
                   "status": st}

    def vcycle_solve(self, b, x=None, rtol=1e-9, maxit=500, raise_on_fail=True):
        """The V-cycle as a stand-alone iterative solver (cmg_vcycle_solve)."""
        x = self._empty(None) if x is None else x
        n = self.ndofs(None)
        info = SolveInfo()
        st = _lib.cmg_vcycle_solve(self._h, _dev(b, n), _dev(x, n), rtol, maxit, ctypes.byref(info), _stream())
        if raise_on_fail:
            _check(st)
        return x, {"iterations": info.iterations, "rel_residual": info.rel_residual, "n_frac": info.n_frac,
                   "status": st}

    def vcycle_multi(self, r, z=None):
        """z[c] = B r[c] for the rows c of r (shape (nrhs, n), nrhs <= 8)."""
        import torch

        nrhs, n = r.shape
        if n != self.ndofs(None):
            raise ValueError("columns must have the finest level's length")
        z = torch.empty_like(r) if z is None else z
        _check(_lib.cmg_vcycle_multi(self._h, nrhs, _dev(r, nrhs * n), _dev(z, nrhs * n), _stream()))
        return z

    def solve_multi(self, b, x=None, rtol=1e-8, maxit=200, raise_on_fail=True):
        """PCG for every row of b (shape (nrhs, n)); returns x and one info dict per row."""
        import torch

        nrhs, n = b.shape
        if n != self.ndofs(None):
            raise ValueError("columns must have the finest level's length")
        x = torch.empty_like(b) if x is None else x
        info = (SolveInfo * nrhs)()
        st = _lib.cmg_solve_multi(self._h, nrhs, _dev(b, nrhs * n), _dev(x, nrhs * n), rtol, maxit, info, _stream())
        if raise_on_fail:
            _check(st)
        return x, [{"iterations": i.iterations, "rel_residual": i.rel_residual, "n_frac": i.n_frac, "status": st}
                   for i in info]

    def rhs_manufactured(self) -> np.ndarray:
        b = np.empty(self.ndofs(None), dtype=np.float64)
        _check(_lib.cmg_rhs_manufactured(self._h, b.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return b

    def rhs_fourier(self, kappa, amp, phase) -> np.ndarray:
        """Load vector of f = sum_q amp_q cos(pi kappa_q . x + phase_q), g = 0 (host array)."""
        kappa = np.ascontiguousarray(kappa, dtype=np.int32)
        amp = np.ascontiguousarray(amp, dtype=np.float64)
        phase = np.ascontiguousarray(phase, dtype=np.float64)
        b = np.empty(self.ndofs(None), dtype=np.float64)
        _check(_lib.cmg_rhs_fourier(self._h, len(amp), kappa.ctypes.data_as(ctypes.c_void_p),
                                    amp.ctypes.data_as(ctypes.c_void_p), phase.ctypes.data_as(ctypes.c_void_p),
                                    b.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return b

    def rhs_fourier_device(self, kappa, amp, phase, b=None):
        """The same load vector assembled on the device (cmg_rhs_fourier_device)
        into b (a float64 CUDA tensor, allocated when not given)."""
        import torch

        kappa = np.ascontiguousarray(kappa, dtype=np.int32)
        amp = np.ascontiguousarray(amp, dtype=np.float64)
        phase = np.ascontiguousarray(phase, dtype=np.float64)
        n = self.ndofs(None)
        if b is None:
            b = torch.empty(n, dtype=torch.float64, device="cuda")
        _check(_lib.cmg_rhs_fourier_device(self._h, len(amp), kappa.ctypes.data_as(ctypes.c_void_p),
                                           amp.ctypes.data_as(ctypes.c_void_p),
                                           phase.ctypes.data_as(ctypes.c_void_p), _dev(b, n), _stream()))
        return b

    def export(self, level, what: int, dtype) -> np.ndarray:
        level = self._lvl(level)
        need = ctypes.c_size_t()
        _check(_lib.cmg_export(self._h, level, what, None, 0, ctypes.byref(need)))
        out = np.empty(need.value // np.dtype(dtype).itemsize, dtype=dtype)
        if need.value:
            _check(_lib.cmg_export(self._h, level, what, out.ctypes.data_as(ctypes.c_void_p), need.value,
                                   ctypes.byref(need)))
        return out

    KERNEL_KINDS = {"apply": 0, "interior_step": 1, "cut_solve": 2, "cut_update": 3, "prolong": 4,
                    "restrict": 5, "coarse": 6, "layout": 7, "vector": 8}

    def timing(self, kinds=(), level: int = None):
        """Bracket the launches of the named kernel kinds with HIP events (empty:
        off), on every level or only on `level`."""
        mask = 0
        for k in kinds:
            mask |= 1 << self.KERNEL_KINDS[k]
        if mask and level is not None:
            mask |= (level + 1) << 16
        _check(_lib.cmg_timing(self._h, mask))

    def timing_read(self, kind: str, level: int = -1):
        """(launches, total ms) of one kernel kind since the last timing() call."""
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        _check(_lib.cmg_timing_read(self._h, self.KERNEL_KINDS[kind], level, ctypes.byref(n), ctypes.byref(ms)))
        return n.value, ms.value

    def counts(self, level=None) -> dict:
        v = self.export(level, 0, np.int64)
        keys = ["n_dofs", "active_cells", "cut_cells", "interior_patches", "cut_patches", "sum_nj2",
                "ghost_faces", "nodes_per_dir"]
        return dict(zip(keys, (int(t) for t in v)))


class Group:
    """Grouped V-cycles of several problems of one lattice shape (cmg_group_*)."""

    def __init__(self, problems):
        load_library()
        self.problems = list(problems)
        arr = (ctypes.c_void_p * len(self.problems))(*[p._h for p in self.problems])
        h = ctypes.c_void_p()
        _check(_lib.cmg_group_create(arr, len(self.problems), ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _lib.cmg_group_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _ptrs(self, ts):
        if len(ts) != len(self.problems):
            raise ValueError("one vector per member")
        return (ctypes.c_void_p * len(ts))(*[_dev(t, p.ndofs(None)).value for t, p in zip(ts, self.problems)])

    def vcycle(self, rs, zs=None):
        """zs[m] = B_m rs[m] for every member."""
        import torch

        zs = [torch.empty_like(r) for r in rs] if zs is None else zs
        _check(_lib.cmg_group_vcycle(self._h, self._ptrs(rs), self._ptrs(zs), _stream()))
        return zs

    def solve(self, bs, xs=None, rtol=1e-8, maxit=200, raise_on_fail=True):
        """One PCG per member with grouped V-cycles; returns the solutions and one info dict per member."""
        import torch

        xs = [torch.empty_like(b) for b in bs] if xs is None else xs
        g = len(self.problems)
        info = (SolveInfo * g)()
        status = (ctypes.c_int * g)()
        st = _lib.cmg_group_solve(self._h, self._ptrs(bs), self._ptrs(xs), rtol, maxit, info, status, _stream())
        if raise_on_fail:
            _check(st)
        return xs, [{"iterations": i.iterations, "rel_residual": i.rel_residual, "n_frac": i.n_frac, "status": s}
                    for i, s in zip(info, status)]


def footprint(workload, fp32: bool = False, multi: bool = False, quad_n: int = 14):
    """(device bytes, finest-level DoFs) of the problem cmg_setup would build,
    from counts only (cmg_footprint); host only."""
    lib = load_library()
    ls, prm, keep = _levelset_params(workload, quad_n, fp32)
    n = ctypes.c_size_t()
    nd = ctypes.c_int64()
    _check(lib.cmg_footprint(ctypes.byref(ls), ctypes.byref(prm), int(bool(fp32)) | (2 if multi else 0),
                             ctypes.byref(n), ctypes.byref(nd)))
    del keep
    return n.value, nd.value


def _levelset_params(workload, quad_n=14, fp32=False):
    d = workload.dim
    centers = (ctypes.c_double * (len(workload.centers) * d))(*[v for c in workload.centers for v in c])
    semi = (ctypes.c_double * (len(workload.semi) * d))(*[v for s in workload.semi for v in s])
    ls = LevelSet(d, len(workload.centers), centers, semi, workload.lo, workload.hi)
    prm = _params(workload, quad_n, fp32)
    return ls, prm, (centers, semi)


def _params(workload, quad_n=14, fp32=False):
    gm = (ctypes.c_double * 3)(*(list(workload.gamma_m) + [0.0] * 3)[:3])
    return Params(workload.k, workload.n_levels, workload.coarse_cells, workload.gamma_D, workload.gamma_g,
                  workload.ghost_exp_mode, workload.n_c, quad_n, int(bool(fp32)), gm)


class Server:
    """Continuous-batching solve server of the library (one GPU, max_slots
    concurrent solves, admission by device footprint, resident hierarchies)."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int):
        load_library()
        h = ctypes.c_void_p()
        st = _lib.cmg_server_create(int(hbm_budget_bytes), int(max_slots), ctypes.byref(h))
        if st != 0:
            raise CutmgError(st, "server creation failed")
        self._h = h
        self._keep = {}

    def submit(self, workload, fourier=None, rtol=1e-8, maxit=200, fp32=True, quad_n=14) -> int:
        """Queue one solve; fourier = (kappa, amp, theta) or None for the manufactured problem."""
        ls, prm, keep = _levelset_params(workload, quad_n, fp32)
        arrays = []
        if fourier is not None:
            kappa = np.ascontiguousarray(fourier[0], dtype=np.int32)
            amp = np.ascontiguousarray(fourier[1], dtype=np.float64)
            theta = np.ascontiguousarray(fourier[2], dtype=np.float64)
            arrays = [kappa, amp, theta]
            req = Request(ls, prm, len(amp), kappa.ctypes.data, amp.ctypes.data, theta.ctypes.data, rtol, maxit)
        else:
            req = Request(ls, prm, 0, None, None, None, rtol, maxit)
        t = ctypes.c_uint64()
        st = _lib.cmg_submit(self._h, ctypes.byref(req), ctypes.byref(t))
        if st != 0:
            raise CutmgError(st, "submit failed")
        del keep, arrays  # the request is copied by the library
        return t.value

    def poll(self, ticket: int, n_dofs: int = None):
        """None while pending, else (result dict, solution or None)."""
        res = Result()
        x = None
        if n_dofs is not None:
            x = np.empty(n_dofs, dtype=np.float64)
        st = _lib.cmg_poll(self._h, ticket, ctypes.byref(res), x.ctypes.data if x is not None else None,
                           n_dofs if n_dofs is not None else 0)
        if st == CMG_PENDING:
            return None
        if st == CMG_EINVAL and x is not None:
            # no solution of that length: a failed request keeps none
            st = _lib.cmg_poll(self._h, ticket, ctypes.byref(res), None, 0)
            x = None
        if st != 0:
            raise CutmgError(st, "poll failed")
        out = {"status": res.status, "n_dofs": res.n_dofs, "iterations": res.info.iterations,
               "rel_residual": res.info.rel_residual, "cache_hit": bool(res.cache_hit),
               "t_submit": res.t_submit, "t_start": res.t_start, "t_admitted": res.t_admitted,
               "t_solve_start": res.t_solve_start, "t_done": res.t_done, "batch": res.batch,
               "group": res.group}
        return out, x

    def close(self):
        if getattr(self, "_h", None):
            _lib.cmg_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
