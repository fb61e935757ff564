"""Python binding of the MI355X wave-propagation library (libwavepatch.so).

Argument marshalling only: every step of the hot path runs in the HIP
kernels behind the C ABI declared in include/wp.h.  PyTorch supplies device
memory (through the library's allocator hook) and the HIP stream.  There is
no CPU fallback: if the shared library is missing, importing ``lib()``
raises.

Names follow the C ABI: ``WavePatch.step_patches`` is ``wp_step_patches``,
``adjoint_run`` is ``wp_adjoint_run``, ``flag_adjoint`` is
``wp_flag_adjoint``, ``regrid`` is ``wp_regrid`` and so on.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwavepatch.so")

WP_OK, WP_EINVAL, WP_ENOMEM, WP_EDEVICE, WP_ECFL, WP_ENONFINITE, WP_ERANGE, WP_ESTATE = 0, -1, -2, -3, -4, -5, -6, -7
ACOUSTICS_1D, ACOUSTICS_2D, SWE_2D = 1, 2, 3
BC_EXTRAP, BC_WALL, BC_PERIODIC = 0, 1, 2
FP64, FP32, MIXED = 64, 32, 16
FUNC_INTERVAL, FUNC_BOX, FUNC_DISC = 0, 1, 2
MAX_LEVELS = 6


class WPError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


class wp_problem(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("bc", ctypes.c_int * 4), ("order", ctypes.c_int),
                ("limiter", ctypes.c_int), ("transverse", ctypes.c_int), ("precision", ctypes.c_int),
                ("cfl_max", ctypes.c_double), ("g", ctypes.c_double)]


class wp_coefficients(ctypes.Structure):
    _fields_ = [("rho", ctypes.POINTER(ctypes.c_double)), ("K", ctypes.POINTER(ctypes.c_double)),
                ("B", ctypes.POINTER(ctypes.c_double))]


class wp_grid(ctypes.Structure):
    _fields_ = [("xlo", ctypes.c_double), ("xhi", ctypes.c_double), ("ylo", ctypes.c_double),
                ("yhi", ctypes.c_double), ("nx0", ctypes.c_int), ("ny0", ctypes.c_int),
                ("num_levels", ctypes.c_int), ("ratio", ctypes.c_int * MAX_LEVELS)]


class wp_patch(ctypes.Structure):
    _fields_ = [("ilo", ctypes.c_int), ("jlo", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int)]


class wp_functional(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("component", ctypes.c_int), ("x0", ctypes.c_double),
                ("x1", ctypes.c_double), ("y0", ctypes.c_double), ("y1", ctypes.c_double),
                ("cx", ctypes.c_double), ("cy", ctypes.c_double), ("r", ctypes.c_double)]


class wp_snapshot_spec(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("nsteps", ctypes.c_int), ("snap_every", ctypes.c_int)]


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class wp_allocator(ctypes.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("user", ctypes.c_void_p)]


# every symbol include/wp.h declares, with its ctypes signature
_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
_SIGS = {
    "wp_create": (_I, [ctypes.POINTER(wp_problem), ctypes.POINTER(wp_coefficients), ctypes.POINTER(wp_grid),
                       ctypes.POINTER(wp_allocator), _P, ctypes.POINTER(_P)]),
    "wp_destroy": (None, [_P]),
    "wp_last_error": (ctypes.c_char_p, [_P]),
    "wp_status_string": (ctypes.c_char_p, [_I]),
    "wp_set_stream": (_I, [_P, _P]),
    "wp_set_bathymetry": (_I, [_P, _I, ctypes.POINTER(_D)]),
    "wp_level_info": (_I, [_P, _I, ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_I)]),
    "wp_set_state": (_I, [_P, _I, _I, _P, _I]),
    "wp_get_state": (_I, [_P, _I, _I, _P, _I]),
    "wp_step_patches": (_I, [_P, _I, _D]),
    "wp_advance": (_I, [_P, _I, _D]),
    "wp_set_equation": (_I, [_P, _I]),
    "wp_set_snapshots": (_I, [_P, _P, _I, _D, _I]),
    "wp_get_equation": (_I, [_P, ctypes.POINTER(_I)]),
    "wp_set_reflux": (_I, [_P, _I]),
    "wp_get_reflux": (_I, [_P, ctypes.POINTER(_I)]),
    "wp_adjoint_run": (_I, [_P, ctypes.POINTER(wp_functional), ctypes.POINTER(wp_snapshot_spec)]),
    "wp_num_snapshots": (_I, [_P]),
    "wp_get_snapshot": (_I, [_P, _I, _P, _I]),
    "wp_flag_adjoint": (_I, [_P, _I, _D, _D, _D, _D, _P, _I, ctypes.POINTER(ctypes.c_int64)]),
    "wp_flag_difference": (_I, [_P, _I, _D, _P, _I, ctypes.POINTER(ctypes.c_int64)]),
    "wp_flag_surface": (_I, [_P, _I, _D, _P, _I, ctypes.POINTER(ctypes.c_int64)]),
    "wp_flag_richardson": (_I, [_P, _I, _D, _I, _D, _D, _D, _D, _P, _I, ctypes.POINTER(ctypes.c_int64),
                                ctypes.POINTER(_D)]),
    "wp_regrid": (_I, [_P, _I, ctypes.POINTER(wp_patch), _I, _I]),
    "wp_get_patches": (_I, [_P, _I, ctypes.POINTER(wp_patch), _I, ctypes.POINTER(_I)]),
    "wp_get_flags": (_I, [_P, _I, _P, _I]),
    "wp_forward_flagged": (_I, [_P, _D, _I, _I, _D, _D, _D, ctypes.POINTER(ctypes.c_int64),
                                ctypes.POINTER(ctypes.c_float)]),
    "wp_cluster": (_I, [_P, _P, _I, _I, _D, _I, _I, ctypes.POINTER(wp_patch), _I, ctypes.POINTER(_I)]),
    "wp_inner_product_noalloc": (_I, [_P, _P, _I, ctypes.c_longlong, _I, _D, _P, _P]),
    "wp_functional_value": (_I, [_P, ctypes.POINTER(wp_functional), _I, _I, ctypes.POINTER(_D)]),
    "wp_get_time": (_I, [_P, _I, ctypes.POINTER(_D)]),
    "wp_set_time": (_I, [_P, _I, _D]),
    "wp_sync": (_I, [_P]),
    "wp_host_times": (_I, [_P, ctypes.POINTER(_D), _I, _I]),
    "wp_batch_create": (_I, [ctypes.POINTER(_P), _I, ctypes.POINTER(_D), ctypes.POINTER(_P)]),
    "wp_batch_destroy": (None, [_P]),
    "wp_batch_step": (_I, [_P, _I, _I]),
    "wp_batch_adjoint_run": (_I, [_P, ctypes.POINTER(wp_functional), _I, _I]),
    "wp_batch_last_error": (ctypes.c_char_p, [_P]),
    "wp_set_tile_rows": (_I, [_P, _I]),
    "wp_set_step_pairs": (_I, [_P, _I]),
    "wp_get_step_pairs": (_I, [_P, ctypes.POINTER(_I)]),
    "wp_get_tile_rows": (_I, [_P, ctypes.POINTER(_I)]),
    "wp_run_graph": (_I, [_P, _I, _D, _I]),
}

_lib = None


def lib():
    """Load libwavepatch.so (built by ``paper_1511_03645_amd.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1511_03645_amd.build`")
        # PyTorch's HIP runtime is loaded first, so that the library binds to
        # the runtime that owns the device memory and streams torch hands it
        _torch()
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _torch():
    try:
        import torch
        return torch
    except Exception:          # pragma: no cover
        return None


class CallbackAllocator:
    """wp_allocator from two Python callables: alloc(nbytes) -> device
    address or None, free(address)."""

    def __init__(self, alloc, free):
        def _alloc(nbytes, user):
            p = alloc(int(nbytes))
            return p if p else None

        def _free(p, user):
            free(p)

        self._a = _ALLOC_FN(_alloc)
        self._f = _FREE_FN(_free)
        self.struct = wp_allocator(self._a, self._f, None)


class TorchAllocator:
    """wp_allocator backed by the PyTorch caching allocator on one device."""

    def __init__(self, device="cuda"):
        torch = _torch()
        self.device = device
        self.blocks = {}

        def _alloc(nbytes, user):
            try:
                t = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
            except Exception:
                return None
            p = t.data_ptr()
            self.blocks[p] = t
            return p

        def _free(p, user):
            self.blocks.pop(p, None)

        self._a = _ALLOC_FN(_alloc)
        self._f = _FREE_FN(_free)
        self.struct = wp_allocator(self._a, self._f, None)


def functional_struct(f):
    kinds = {"interval": FUNC_INTERVAL, "box": FUNC_BOX, "disc": FUNC_DISC}
    return wp_functional(kinds[f["kind"]], int(f.get("component", 0)), f.get("x0", 0.0), f.get("x1", 0.0),
                         f.get("y0", 0.0), f.get("y1", 0.0), f.get("cx", 0.0), f.get("cy", 0.0), f.get("r", 0.0))


def cluster(flags, allowed=None, efficiency=0.7, maxside=16, minside=2):
    """Berger-Rigoutsos boxes (ilo, jlo, nx, ny) of a [ny][nx] flag image
    (``wp_cluster``; host only)."""
    f = np.ascontiguousarray(flags, dtype=np.uint8)
    ny, nx = f.shape
    a = None if allowed is None else np.ascontiguousarray(allowed, dtype=np.uint8)
    if a is not None and a.shape != f.shape:
        raise ValueError("allowed must match flags")
    n = ctypes.c_int()
    args = (f.ctypes.data, None if a is None else a.ctypes.data, nx, ny, float(efficiency), int(maxside), int(minside))
    rc = lib().wp_cluster(*args, None, 0, ctypes.byref(n))
    if rc != WP_OK:
        raise WPError(rc, "wp_cluster: " + lib().wp_status_string(rc).decode())
    arr = (wp_patch * max(1, n.value))()
    rc = lib().wp_cluster(*args, arr, n.value, ctypes.byref(n))
    if rc != WP_OK:
        raise WPError(rc, "wp_cluster: " + lib().wp_status_string(rc).decode())
    return [(p.ilo, p.jlo, p.nx, p.ny) for p in arr[:n.value]]


def inner_product_noalloc(a, b, cells, m, dA, out, precision=FP64, stream=None):
    """wp_inner_product_noalloc on torch device tensors: out (one float64 on
    the device) = dA * sum_k sum_i a_k[i] b_k[i]; a, b [m][cells] contiguous,
    float64 (FP64) or float32 (FP32).  Enqueued on `stream` (default: torch's
    current stream); nothing is allocated by the library."""
    torch = _torch()
    for t in (a, b, out):
        if not (t.is_cuda and t.is_contiguous()):
            raise ValueError("a, b and out must be contiguous device tensors")
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    rc = lib().wp_inner_product_noalloc(ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()), precision,
                                        int(cells), int(m), float(dA), ctypes.c_void_p(out.data_ptr()),
                                        ctypes.c_void_p(stream or 0))
    if rc != WP_OK:
        raise WPError(rc, "wp_inner_product_noalloc: " + lib().wp_status_string(rc).decode())


def _ptr(a):
    """(pointer, on_device) of a numpy array or torch tensor."""
    torch = _torch()
    if torch is not None and isinstance(a, torch.Tensor):
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return ctypes.c_void_p(a.data_ptr()), int(a.is_cuda)
    if not a.flags["C_CONTIGUOUS"]:
        raise ValueError("array must be C-contiguous")
    return ctypes.c_void_p(a.ctypes.data), 0


class WavePatch:
    """One solver instance (a wp_ctx)."""

    def __init__(self, kind, nx, ny=1, xlo=0.0, xhi=1.0, ylo=0.0, yhi=1.0, rho=None, K=None, B=None,
                 bc=(BC_EXTRAP,) * 4, order=2, limiter=1, transverse=1, precision=FP64, cfl_max=1.0, g=9.81,
                 num_levels=1, ratios=(), stream=None, torch_alloc=True, allocator=None):
        L = lib()
        kinds = {"acoustics1d": ACOUSTICS_1D, "acoustics2d": ACOUSTICS_2D, "swe2d": SWE_2D}
        self.kind = kind
        self.kind_id = kinds[kind] if isinstance(kind, str) else kind
        self.precision = precision
        self.m = 2 if self.kind_id == ACOUSTICS_1D else 3
        prob = wp_problem(self.kind_id, (ctypes.c_int * 4)(*bc), order, limiter, transverse, precision, cfl_max, g)
        self._keep = []

        def dptr(a):
            if a is None:
                return ctypes.POINTER(ctypes.c_double)()
            a = np.ascontiguousarray(a, dtype=np.float64)
            self._keep.append(a)
            return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        coef = wp_coefficients(dptr(rho), dptr(K), dptr(B))
        rat = (ctypes.c_int * MAX_LEVELS)(*(list(ratios) + [1] * (MAX_LEVELS - len(ratios))))
        grid = wp_grid(xlo, xhi, ylo, yhi, nx, ny if self.kind_id != ACOUSTICS_1D else 1, num_levels, rat)
        torch = _torch()
        self.allocator = allocator
        alloc_p = None if allocator is None else ctypes.byref(allocator.struct)
        if torch is not None and torch.cuda.is_available():
            if stream is None:
                stream = torch.cuda.current_stream().cuda_stream
            if torch_alloc and allocator is None:
                self.allocator = TorchAllocator()
                alloc_p = ctypes.byref(self.allocator.struct)
        self.stream = stream
        h = ctypes.c_void_p()
        rc = L.wp_create(ctypes.byref(prob), ctypes.byref(coef), ctypes.byref(grid), alloc_p,
                         ctypes.c_void_p(stream or 0), ctypes.byref(h))
        self._keep = []
        if rc != WP_OK:
            msg = L.wp_last_error(h).decode() if h.value else L.wp_status_string(rc).decode()
            if h.value:
                L.wp_destroy(h)
            raise WPError(rc, msg)
        self.h = h
        self.nx, self.ny = nx, (ny if self.kind_id != ACOUSTICS_1D else 1)

    # -- plumbing ---------------------------------------------------------
    def _check(self, rc):
        if rc != WP_OK:
            raise WPError(rc, lib().wp_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().wp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_bathymetry(self, level, B):
        """wp_set_bathymetry: cell averages [ny_l][nx_l] of a refined shallow-water level."""
        B = np.ascontiguousarray(B, dtype=np.float64)
        self._check(lib().wp_set_bathymetry(self.h, level, B.ctypes.data_as(ctypes.POINTER(_D))))

    def level_info(self, level):
        nx, ny, npch = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        self._check(lib().wp_level_info(self.h, level, ctypes.byref(nx), ctypes.byref(ny), ctypes.byref(npch)))
        return nx.value, ny.value, npch.value

    def _dtypes(self):
        if self.precision == FP64:
            return [np.float64] * self.m
        if self.precision == FP32:
            return [np.float32] * self.m
        return [np.float64, np.float32, np.float32]

    def _box(self, level, patch):
        if patch < 0:
            nx, ny, _ = self.level_info(level)
            return nx, ny
        p = self.get_patches(level)[patch]
        return p[2], p[3]

    def _pack(self, q):
        """Pack [m][ny][nx] into the library's byte layout for this precision."""
        dts = self._dtypes()
        return np.concatenate([np.ascontiguousarray(q[k], dtype=dts[k]).ravel().view(np.uint8) for k in range(self.m)])

    def _unpack(self, buf, nx, ny):
        dts = self._dtypes()
        out, off = [], 0
        for k in range(self.m):
            nb = nx * ny * np.dtype(dts[k]).itemsize
            out.append(buf[off:off + nb].view(dts[k]).reshape(ny, nx).astype(np.float64))
            off += nb
        return np.stack(out)

    # -- C ABI ------------------------------------------------------------
    def set_state(self, q, level=0, patch=-1):
        """wp_set_state: q is [m][ny][nx] (numpy, any float type), or a device
        tensor already in the library's byte layout."""
        torch = _torch()
        if torch is not None and isinstance(q, torch.Tensor) and q.is_cuda:
            p, dev = _ptr(q)
        else:
            nx, ny = self._box(level, patch)
            q = np.asarray(q).reshape(self.m, ny, nx)
            buf = self._pack(q)
            p, dev = _ptr(buf)
        self._check(lib().wp_set_state(self.h, level, patch, p, dev))

    def get_state(self, level=0, patch=-1):
        """wp_get_state into a host [m][ny][nx] float64 array."""
        nx, ny = self._box(level, patch)
        itemsizes = [np.dtype(d).itemsize for d in self._dtypes()]
        buf = np.empty(nx * ny * sum(itemsizes), dtype=np.uint8)
        p, dev = _ptr(buf)
        self._check(lib().wp_get_state(self.h, level, patch, p, dev))
        return self._unpack(buf, nx, ny)

    def step_patches(self, level, dt):
        self._check(lib().wp_step_patches(self.h, level, dt))

    def advance(self, nsteps, dt0):
        self._check(lib().wp_advance(self.h, nsteps, dt0))

    def set_equation(self, adjoint):
        """Solve the adjoint system (True) or the forward system (False) in
        the hierarchy's steps."""
        self._check(lib().wp_set_equation(self.h, 1 if adjoint else 0))

    def get_equation(self):
        v = ctypes.c_int(0)
        self._check(lib().wp_get_equation(self.h, ctypes.byref(v)))
        return bool(v.value)

    def set_reflux(self, on):
        """wp_set_reflux: flux correction at coarse-fine edges of the adjoint
        acoustics hierarchy or of the shallow-water hierarchy."""
        self._check(lib().wp_set_reflux(self.h, int(on)))

    def get_reflux(self):
        v = ctypes.c_int()
        self._check(lib().wp_get_reflux(self.h, ctypes.byref(v)))
        return bool(v.value)

    def adjoint_run(self, functional, dt, nsteps, snap_every):
        f = functional_struct(functional)
        sp = wp_snapshot_spec(dt, nsteps, snap_every)
        self._check(lib().wp_adjoint_run(self.h, ctypes.byref(f), ctypes.byref(sp)))

    def num_snapshots(self):
        return lib().wp_num_snapshots(self.h)

    def set_snapshots(self, snaps, ds):
        """Install a snapshot store: snaps [nsnap, m, ny0, nx0] (the store's
        precision: FP64 for FP64 problems, else FP32), snapshot n at adjoint
        time n * ds."""
        nx, ny, _ = self.level_info(0)
        dt = np.float64 if self.precision == FP64 else np.float32
        a = np.ascontiguousarray(snaps, dtype=dt)
        if a.ndim != 4 or a.shape[1:] != (self.m, ny, nx):
            raise ValueError(f"snapshots must be [nsnap, {self.m}, {ny}, {nx}], got {a.shape}")
        p, dev = _ptr(a)
        self._check(lib().wp_set_snapshots(self.h, p, a.shape[0], float(ds), dev))

    def get_snapshot(self, n):
        nx, ny, _ = self.level_info(0)
        es = 8 if self.precision == FP64 else 4
        buf = np.empty(self.m * nx * ny * es, dtype=np.uint8)
        p, dev = _ptr(buf)
        self._check(lib().wp_get_snapshot(self.h, n, p, dev))
        return buf.view(np.float64 if es == 8 else np.float32).reshape(self.m, ny, nx).astype(np.float64)

    def flag_adjoint(self, level, tol, t, t_s, t_f, want_flags=True, want_count=True):
        """wp_flag_adjoint; with want_flags and want_count False nothing is
        copied back and the call does not synchronise."""
        nx, ny, _ = self.level_info(level)
        flags = np.zeros((ny, nx), dtype=np.uint8) if want_flags else None
        n = ctypes.c_int64()
        p = ctypes.c_void_p(flags.ctypes.data) if want_flags else ctypes.c_void_p()
        self._check(lib().wp_flag_adjoint(self.h, level, tol, t, t_s, t_f, p, 0,
                                          ctypes.byref(n) if want_count else None))
        return flags, (n.value if want_count else None)

    def _flag_standard(self, fn, level, tol, want_flags, want_count):
        nx, ny, _ = self.level_info(level)
        flags = np.zeros((ny, nx), dtype=np.uint8) if want_flags else None
        n = ctypes.c_int64()
        p = ctypes.c_void_p(flags.ctypes.data) if want_flags else ctypes.c_void_p()
        self._check(fn(self.h, level, tol, p, 0, ctypes.byref(n) if want_count else None))
        return flags, (n.value if want_count else None)

    def flag_difference(self, level, tol, want_flags=True, want_count=True):
        """wp_flag_difference (undivided differences of every component)."""
        return self._flag_standard(lib().wp_flag_difference, level, tol, want_flags, want_count)

    def flag_surface(self, level, tol, want_flags=True, want_count=True):
        """wp_flag_surface (shallow water: |eta| above sea level 0)."""
        return self._flag_standard(lib().wp_flag_surface, level, tol, want_flags, want_count)

    def flag_richardson(self, dt, tol, weighted=False, t=0.0, t_s=0.0, t_f=0.0, level=0, want_flags=True,
                        want_count=True, want_estimate=False):
        """wp_flag_richardson: (flags, count, estimate [m][ny/2][nx/2] or None)."""
        nx, ny, _ = self.level_info(level)
        flags = np.zeros((ny, nx), dtype=np.uint8) if want_flags else None
        est = np.zeros((self.m, ny // 2, nx // 2)) if want_estimate else None
        n = ctypes.c_int64()
        p = ctypes.c_void_p(flags.ctypes.data) if want_flags else ctypes.c_void_p()
        e = est.ctypes.data_as(ctypes.POINTER(_D)) if want_estimate else None
        self._check(lib().wp_flag_richardson(self.h, level, dt, int(weighted), tol, t, t_s, t_f, p, 0,
                                             ctypes.byref(n) if want_count else None, e))
        return flags, (n.value if want_count else None), est

    def get_flags(self, level=0):
        """wp_get_flags: the level's flag canvas [ny][nx] (uint8) as the last
        flag call on it left it."""
        nx, ny, _ = self.level_info(level)
        flags = np.zeros((ny, nx), dtype=np.uint8)
        self._check(lib().wp_get_flags(self.h, level, ctypes.c_void_p(flags.ctypes.data), 0))
        return flags

    def forward_flagged(self, dt, nsteps, flag_every, tol, t_s, t_f, want_counts=True, want_times=False):
        """wp_forward_flagged: (flagged cells per flag event or None,
        duration in ms of the first step launch of each block or None)."""
        nev = nsteps // flag_every if flag_every > 0 else 0
        counts = (ctypes.c_int64 * max(1, nev))() if want_counts else None
        times = (ctypes.c_float * max(1, nev))() if want_times else None
        self._check(lib().wp_forward_flagged(self.h, dt, nsteps, flag_every, tol, t_s, t_f, counts, times))
        return (list(counts[:nev]) if want_counts else None), (list(times[:nev]) if want_times else None)

    def regrid(self, level, patches=None, buffer=0):
        if patches is None:
            self._check(lib().wp_regrid(self.h, level, None, 0, buffer))
        else:
            arr = (wp_patch * max(1, len(patches)))(*[wp_patch(*map(int, p)) for p in patches])
            self._check(lib().wp_regrid(self.h, level, arr, len(patches), buffer))

    def get_patches(self, level):
        n = ctypes.c_int()
        self._check(lib().wp_get_patches(self.h, level, None, 0, ctypes.byref(n)))
        arr = (wp_patch * max(1, n.value))()
        self._check(lib().wp_get_patches(self.h, level, arr, n.value, ctypes.byref(n)))
        return [(p.ilo, p.jlo, p.nx, p.ny) for p in arr[:n.value]]

    def functional_value(self, functional, which=0, snapshot=0):
        f = functional_struct(functional)
        out = ctypes.c_double()
        self._check(lib().wp_functional_value(self.h, ctypes.byref(f), which, snapshot, ctypes.byref(out)))
        return out.value

    def get_time(self, level=0):
        t = ctypes.c_double()
        self._check(lib().wp_get_time(self.h, level, ctypes.byref(t)))
        return t.value

    def set_time(self, t, level=0):
        self._check(lib().wp_set_time(self.h, level, t))

    def host_times(self, reset=False):
        """wp_host_times: dict of cumulative host milliseconds (flag copy,
        clustering, table rebuild and upload, capture, the upload's
        host-to-device copies, tile-table rebuilds) and capture counts."""
        v = (_D * 8)()
        self._check(lib().wp_host_times(self.h, v, 8, int(reset)))
        keys = ("flag_copy_ms", "cluster_ms", "upload_ms", "capture_ms", "captures", "graph_updates", "h2d_ms",
                "tiles_ms")
        return dict(zip(keys, list(v)))

    def sync(self):
        self._check(lib().wp_sync(self.h))

    def set_tile_rows(self, rows):
        self._check(lib().wp_set_tile_rows(self.h, rows))

    def get_tile_rows(self):
        r = ctypes.c_int()
        self._check(lib().wp_get_tile_rows(self.h, ctypes.byref(r)))
        return r.value

    def set_step_pairs(self, rows):
        """Two steps per launch in graph, adjoint and flagged runs: rows -1
        (built-in tile height), 0 (off), or 4 to 64 rows per tile."""
        self._check(lib().wp_set_step_pairs(self.h, rows))

    def get_step_pairs(self):
        r = ctypes.c_int()
        self._check(lib().wp_get_step_pairs(self.h, ctypes.byref(r)))
        return r.value

    def run_graph(self, nsteps, dt, replays):
        self._check(lib().wp_run_graph(self.h, nsteps, dt, replays))


class Batch:
    """wp_batch over independent single-level acoustics instances."""

    def __init__(self, instances, dts):
        self.instances = list(instances)
        arr = (ctypes.c_void_p * len(instances))(*[w.h.value for w in instances])
        d = (ctypes.c_double * len(dts))(*dts)
        h = ctypes.c_void_p()
        rc = lib().wp_batch_create(arr, len(instances), d, ctypes.byref(h))
        if rc != WP_OK:
            raise WPError(rc, lib().wp_batch_last_error(h).decode() if h.value else "batch creation failed")
        self.h = h

    def _check(self, rc):
        if rc != WP_OK:
            raise WPError(rc, lib().wp_batch_last_error(self.h).decode())

    def step(self, nsteps, adjoint=False):
        self._check(lib().wp_batch_step(self.h, nsteps, int(adjoint)))

    def adjoint_run(self, functionals, nsteps, snap_every):
        arr = (wp_functional * len(functionals))(*[functional_struct(f) for f in functionals])
        self._check(lib().wp_batch_adjoint_run(self.h, arr, nsteps, snap_every))

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().wp_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def from_config(cfg, precision=FP64, num_levels=1, ratios=(), **kw):
    """Instance for a workload dict of ``wp_synth`` (argument marshalling)."""
    kind = cfg["kind"]
    args = dict(kind=kind, nx=cfg["nx"], ny=cfg.get("ny", 1), xlo=cfg["xlo"], xhi=cfg["xhi"], ylo=cfg["ylo"],
                yhi=cfg["yhi"], bc=tuple(cfg["bc"]), order=cfg["order"], limiter=cfg["limiter"],
                transverse=cfg["transverse"], precision=precision, num_levels=num_levels, ratios=ratios,
                g=cfg.get("g", 9.81))
    if kind == "swe2d":
        args["B"] = cfg["B"]
    else:
        args["rho"] = cfg["rho"]
        args["K"] = cfg["K"]
    args.update(kw)
    return WavePatch(**args)
