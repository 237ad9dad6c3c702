"""ctypes binding of libtopo (include/topo.h): argument marshalling only.

Every numerical step runs in the HIP library; this module converts Python
problem descriptions and torch device tensors into the C structures and raw
pointers the ABI expects, and turns status codes into exceptions.
"""

from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtopo.so")

TOPO_OK, TOPO_EINVAL, TOPO_ENOMEM, TOPO_EDEVICE, TOPO_ENOTCONVERGED, TOPO_EUNSUPPORTED = range(6)
FILTER_DENSITY, FILTER_SENSITIVITY = 0, 1
VOL_DESIGN, VOL_ALL = 0, 1
FILTER_FWD, FILTER_ADJ, FILTER_SENS, FILTER_VOLW = 0, 1, 2, 3
PREC_FP64, PREC_FP32, PREC_BF16 = 0, 1, 2
PRECOND_JACOBI, PRECOND_MG, PRECOND_LEARNED = 0, 1, 2
KU_AUTO, KU_NODE, KU_ELEMENT = 0, 1, 2
LOSS_REL, LOSS_COS = 0, 1

EXPORTED = [
    "topo_default_opts", "topo_setup", "topo_destroy", "topo_last_error", "topo_sizes",
    "topo_apply_K", "topo_apply_precond", "topo_solve", "topo_sensitivity", "topo_filter", "topo_oc_update",
    "topo_iterate", "topo_get_state", "topo_time_operator",
    "topo_nn_create", "topo_nn_destroy", "topo_nn_set_precision", "topo_nn_n_params", "topo_nn_set_weights", "topo_nn_get_weights",
    "topo_nn_forward", "topo_nn_loss_grad", "topo_default_train_opts", "topo_nn_train", "topo_set_nn",
    "topo_nn_make_pairs", "topo_setup_batch", "topo_destroy_batch", "topo_batch_context", "topo_iterate_batch",
    "topo_oc_update_noalloc", "topo_surface_stl", "topo_voxelize", "topo_clear_tuning_cache",
]
_VOID = ("topo_default_opts", "topo_destroy", "topo_last_error", "topo_nn_destroy", "topo_default_train_opts",
         "topo_destroy_batch", "topo_clear_tuning_cache")


class TopoError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"[status {status}] {msg}")
        self.status = status


class NotConverged(TopoError):
    pass


class Problem_C(C.Structure):
    _fields_ = [
        ("nelx", C.c_int32), ("nely", C.c_int32), ("nelz", C.c_int32),
        ("E0", C.c_double), ("Emin", C.c_double), ("nu", C.c_double), ("penal", C.c_double),
        ("rmin", C.c_double), ("volfrac", C.c_double), ("move", C.c_double), ("eta", C.c_double),
        ("filter", C.c_int32), ("vol_mode", C.c_int32),
        ("mask", C.POINTER(C.c_int8)),
        ("fixed_dofs", C.POINTER(C.c_int64)), ("n_fixed", C.c_int64),
        ("f", C.POINTER(C.c_double)),
    ]


class Opts_C(C.Structure):
    _fields_ = [
        ("precision", C.c_int32), ("precond", C.c_int32), ("mg_levels", C.c_int32),
        ("mg_max_coarse_dof", C.c_int32), ("cheb_degree", C.c_int32), ("cheb_degree_coarse", C.c_int32), ("rtol", C.c_double),
        ("max_iters", C.c_int32), ("warm_start", C.c_int32), ("oc_tol", C.c_double),
        ("check_every", C.c_int32), ("use_graphs", C.c_int32), ("nn_max_iters", C.c_int32),
        ("autotune", C.c_int32), ("coarse_tail_nodes", C.c_int32), ("mfma_smoothing", C.c_int32),
        ("ku_kernel", C.c_int32), ("ku_shape", C.c_int32), ("coarse_refresh", C.c_int32),
        ("cheb_degree_level", C.c_int32 * 8), ("group_launch", C.c_int32),
        ("cheb_upper", C.c_double),
    ]


class SolveStats_C(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("relres", C.c_double),
                ("ms", C.c_double), ("fallbacks", C.c_int32), ("learned_iters", C.c_int32)]


class TrainOpts_C(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_double), ("beta1", C.c_double),
                ("beta2", C.c_double), ("eps", C.c_double), ("seed", C.c_uint64), ("loss", C.c_int32)]


class TrainStats_C(C.Structure):
    _fields_ = [("steps", C.c_int32), ("loss_first", C.c_double), ("loss_last", C.c_double),
                ("ms", C.c_double)]


class IterStats_C(C.Structure):
    _fields_ = [
        ("c", C.c_double), ("volume", C.c_double), ("change", C.c_double), ("lambda_", C.c_double),
        ("pcg_iters", C.c_int32), ("converged", C.c_int32), ("relres", C.c_double),
        ("ms_total", C.c_double), ("ms_filter", C.c_double), ("ms_solve", C.c_double),
        ("ms_sens", C.c_double), ("ms_oc", C.c_double),
        ("fallbacks", C.c_int32), ("learned_iters", C.c_int32),
    ]


_lib = None


def load(path: str = LIB_PATH):
    """Loads libtopo.so; raises if it has not been built (no CPU fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2504_05604_amd.build`")
    # torch brings its own HIP runtime (same soname as the system one); importing
    # it first makes the dynamic loader resolve libtopo's runtime to that same
    # copy, so the process has exactly one HIP runtime and one device context.
    import torch  # noqa: F401
    lib = C.CDLL(path)
    vp, dp = C.c_void_p, C.c_void_p
    lib.topo_default_opts.argtypes = [C.POINTER(Opts_C)]
    lib.topo_default_opts.restype = None
    lib.topo_setup.argtypes = [C.POINTER(Problem_C), C.POINTER(Opts_C), vp, C.POINTER(vp)]
    lib.topo_destroy.argtypes = [vp]
    lib.topo_destroy.restype = None
    lib.topo_last_error.restype = C.c_char_p
    lib.topo_sizes.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int32)]
    lib.topo_apply_K.argtypes = [vp, dp, dp, dp]
    lib.topo_apply_precond.argtypes = [vp, dp, dp, dp]
    lib.topo_solve.argtypes = [vp, dp, dp, C.POINTER(SolveStats_C)]
    lib.topo_sensitivity.argtypes = [vp, dp, dp, dp, dp, C.POINTER(C.c_double)]
    lib.topo_filter.argtypes = [vp, C.c_int32, dp, dp, dp]
    lib.topo_oc_update.argtypes = [vp, dp, dp, dp, dp, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    lib.topo_iterate.argtypes = [vp, dp, C.c_int32, C.POINTER(IterStats_C)]
    lib.topo_get_state.argtypes = [vp, dp, dp]
    lib.topo_time_operator.argtypes = [vp, C.c_int32, C.POINTER(C.c_double)]
    i32p, fp = C.POINTER(C.c_int32), C.c_void_p
    lib.topo_nn_create.argtypes = [i32p, vp, C.POINTER(vp)]
    lib.topo_nn_destroy.argtypes = [vp]
    lib.topo_nn_destroy.restype = None
    lib.topo_nn_n_params.argtypes = [vp, C.POINTER(C.c_int64)]
    lib.topo_nn_set_precision.argtypes = [vp, C.c_int32]
    lib.topo_nn_set_weights.argtypes = [vp, C.POINTER(C.c_float), C.c_int64]
    lib.topo_nn_get_weights.argtypes = [vp, C.POINTER(C.c_float), C.c_int64]
    lib.topo_nn_forward.argtypes = [vp, i32p, C.c_int32, fp, fp]
    lib.topo_nn_loss_grad.argtypes = [vp, i32p, C.c_int64, fp, fp, fp, fp, C.c_int32, i32p, C.c_int32,
                                      C.POINTER(C.c_double), fp]
    lib.topo_default_train_opts.argtypes = [C.POINTER(TrainOpts_C)]
    lib.topo_default_train_opts.restype = None
    lib.topo_nn_train.argtypes = [vp, i32p, C.c_int64, fp, fp, fp, fp, C.POINTER(TrainOpts_C),
                                  C.POINTER(C.c_double), C.POINTER(TrainStats_C)]
    lib.topo_set_nn.argtypes = [vp, vp]
    lib.topo_nn_make_pairs.argtypes = [vp, dp, C.c_int32, i32p, fp, fp, fp, fp]
    lib.topo_setup_batch.argtypes = [C.POINTER(Problem_C), C.c_int32, C.POINTER(Opts_C), C.c_int32, C.POINTER(vp)]
    lib.topo_destroy_batch.argtypes = [vp]
    lib.topo_destroy_batch.restype = None
    lib.topo_batch_context.argtypes = [vp, C.c_int32, C.POINTER(vp)]
    lib.topo_iterate_batch.argtypes = [vp, C.POINTER(vp), C.c_int32, C.POINTER(IterStats_C)]
    lib.topo_surface_stl.argtypes = [C.c_int32, C.c_int32, C.c_int32, dp, C.c_double, C.POINTER(C.c_double),
                                     C.c_double, vp, dp, C.c_int64, C.POINTER(C.c_int64)]
    lib.topo_voxelize.argtypes = [dp, C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_double),
                                  C.c_double, C.c_int8, C.c_int8, vp, dp, C.POINTER(C.c_int64)]
    lib.topo_oc_update_noalloc.argtypes = [C.c_int64, dp, dp, dp, dp, C.c_double, C.c_double, C.c_double,
                                           C.c_double, vp, dp, dp]
    lib.topo_clear_tuning_cache.argtypes = []
    lib.topo_clear_tuning_cache.restype = None
    for name in EXPORTED:
        if name not in _VOID:
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _check(status: int):
    if status == TOPO_OK:
        return
    msg = _lib.topo_last_error().decode()
    if status == TOPO_ENOTCONVERGED:
        raise NotConverged(status, msg)
    raise TopoError(status, msg)


def default_opts(**kw) -> Opts_C:
    lib = load()
    o = Opts_C()
    lib.topo_default_opts(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(f"unknown option {k}")
        if k == "cheb_degree_level":  # per level, finest first; the rest 0 (not set)
            v = list(v) + [0] * (8 - len(v))
            if len(v) != 8:
                raise ValueError("cheb_degree_level takes at most 8 levels")
            v = (C.c_int32 * 8)(*v)
        setattr(o, k, v)
    return o


def _ptr(t, n: Optional[int] = None, dtype=None):
    """Raw device pointer of a contiguous CUDA/HIP tensor (None -> NULL)."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected dtype {dtype}, got {t.dtype}")
    if n is not None and t.numel() != n:
        raise ValueError(f"expected {n} elements, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


def _problem_c(p, filter_mode=None):
    """Problem_C for a problem description, and the host arrays it points to
    (they must stay alive until setup returns; setup copies them)."""
    nel = int(p.nelx * p.nely * p.nelz)
    ndof = int(3 * (p.nelx + 1) * (p.nely + 1) * (p.nelz + 1))
    mask = None if p.mask is None else np.ascontiguousarray(p.mask, dtype=np.int8)
    fixed = np.ascontiguousarray(p.fixed_dofs, dtype=np.int64)
    f = np.ascontiguousarray(p.f, dtype=np.float64)
    if f.size != ndof:
        raise ValueError("load vector has the wrong length")
    if mask is not None and mask.size != nel:
        raise ValueError("mask has the wrong length")
    mode = filter_mode if filter_mode is not None else getattr(p, "filter_mode", "density")
    pc = Problem_C(
        p.nelx, p.nely, p.nelz, p.E0, p.Emin, p.nu, p.penal, p.rmin, p.volfrac, p.move, p.eta,
        FILTER_DENSITY if mode == "density" else FILTER_SENSITIVITY,
        VOL_ALL if getattr(p, "vol_mode", "design") == "all" else VOL_DESIGN,
        None if mask is None else mask.ctypes.data_as(C.POINTER(C.c_int8)),
        fixed.ctypes.data_as(C.POINTER(C.c_int64)), fixed.size,
        f.ctypes.data_as(C.POINTER(C.c_double)),
    )
    return pc, (mask, fixed, f)


def _iter_stats(s) -> dict:
    return {"c": s.c, "volume": s.volume, "change": s.change, "lambda": s.lambda_,
            "pcg_iters": s.pcg_iters, "converged": bool(s.converged), "relres": s.relres,
            "ms_total": s.ms_total, "ms_filter": s.ms_filter, "ms_solve": s.ms_solve,
            "ms_sens": s.ms_sens, "ms_oc": s.ms_oc, "fallbacks": s.fallbacks,
            "learned_iters": s.learned_iters}


class Context:
    """One problem on one device; wraps a topo_ctx."""

    def __init__(self, problem, opts: Optional[Opts_C] = None, stream=None, filter_mode=None):
        lib = load()
        self._lib = lib
        import torch
        # the library shares the process's HIP runtime with torch; let torch create
        # the device context first so both use the same one
        torch.cuda.init()
        self.device = torch.cuda.current_device()
        p = problem
        self.nel = int(p.nelx * p.nely * p.nelz)
        self.ndof = int(3 * (p.nelx + 1) * (p.nely + 1) * (p.nelz + 1))
        pc, self._keep = _problem_c(p, filter_mode)
        self.opts = opts if opts is not None else default_opts()
        handle = C.c_void_p()
        st_ptr = None if stream is None else C.c_void_p(int(stream))
        _check(lib.topo_setup(C.byref(pc), C.byref(self.opts), st_ptr, C.byref(handle)))
        self._h = handle
        lv = C.c_int32()
        _check(lib.topo_sizes(self._h, None, None, C.byref(lv)))
        self.mg_levels = lv.value

    def close(self):
        if getattr(self, "_h", None):
            self._lib.topo_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- entry points ------------------------------------------------------
    def apply_K(self, xphys, u, y):
        import torch
        _check(self._lib.topo_apply_K(self._h, _ptr(xphys, self.nel, torch.float64),
                                      _ptr(u, self.ndof, torch.float64), _ptr(y, self.ndof, torch.float64)))

    def apply_precond(self, xphys, r, z):
        import torch
        _check(self._lib.topo_apply_precond(self._h, _ptr(xphys, self.nel, torch.float64),
                                            _ptr(r, self.ndof, torch.float64), _ptr(z, self.ndof, torch.float64)))

    def solve(self, xphys, u, raise_on_nonconv=True) -> dict:
        import torch
        st = SolveStats_C()
        status = self._lib.topo_solve(self._h, _ptr(xphys, self.nel, torch.float64),
                                      _ptr(u, self.ndof, torch.float64), C.byref(st))
        out = {"iters": st.iters, "converged": bool(st.converged), "relres": st.relres, "ms": st.ms,
               "fallbacks": st.fallbacks, "learned_iters": st.learned_iters}
        if status == TOPO_ENOTCONVERGED and not raise_on_nonconv:
            return out
        _check(status)
        return out

    def sensitivity(self, xphys, u, ce, dc, want_compliance=True):
        import torch
        c = C.c_double()
        _check(self._lib.topo_sensitivity(self._h, _ptr(xphys, self.nel, torch.float64),
                                          _ptr(u, self.ndof, torch.float64), _ptr(ce, self.nel, torch.float64),
                                          _ptr(dc, self.nel, torch.float64),
                                          C.byref(c) if want_compliance else None))
        return c.value if want_compliance else None

    def filter(self, op: int, inp, out, aux=None):
        import torch
        _check(self._lib.topo_filter(self._h, op, _ptr(inp, self.nel, torch.float64),
                                     _ptr(aux, self.nel, torch.float64), _ptr(out, self.nel, torch.float64)))

    def oc_update(self, x, dc, dv, xnew):
        import torch
        chg, lam = C.c_double(), C.c_double()
        _check(self._lib.topo_oc_update(self._h, _ptr(x, self.nel, torch.float64),
                                        _ptr(dc, self.nel, torch.float64), _ptr(dv, self.nel, torch.float64),
                                        _ptr(xnew, self.nel, torch.float64), C.byref(chg), C.byref(lam)))
        return chg.value, lam.value

    def iterate(self, x, n_iter: int, raise_on_nonconv=True) -> List[dict]:
        import torch
        stats = (IterStats_C * max(1, n_iter))()
        status = self._lib.topo_iterate(self._h, _ptr(x, self.nel, torch.float64), n_iter, stats)
        if not (status == TOPO_ENOTCONVERGED and not raise_on_nonconv):
            _check(status)
        return [_iter_stats(stats[i]) for i in range(n_iter)]

    def time_operator(self, reps: int = 50) -> float:
        """Average ms per launch of the finest-level K.u kernel (hipEvents)."""
        ms = C.c_double()
        _check(self._lib.topo_time_operator(self._h, reps, C.byref(ms)))
        return ms.value

    def get_state(self, u=None, xphys=None):
        import torch
        _check(self._lib.topo_get_state(self._h, _ptr(u, self.ndof, torch.float64),
                                        _ptr(xphys, self.nel, torch.float64)))

    def set_nn(self, nn: Optional["Network"]):
        """Attaches a Network as the learned preconditioner (None detaches)."""
        _check(self._lib.topo_set_nn(self._h, None if nn is None else nn._h))
        self._nn = nn  # keep it alive while attached

    def make_pairs(self, xphys, iters, rho, r, e, fixed):
        """Training pairs (r_k, u* - u_k) from CG iterates k in `iters`."""
        import torch
        it = np.ascontiguousarray(iters, dtype=np.int32)
        n = it.size
        V = self.ndof // 3
        _check(self._lib.topo_nn_make_pairs(
            self._h, _ptr(xphys, self.nel, torch.float64), n, it.ctypes.data_as(C.POINTER(C.c_int32)),
            _ptr(rho, n * V, torch.float32), _ptr(r, n * 3 * V, torch.float32),
            _ptr(e, n * 3 * V, torch.float32), _ptr(fixed, n * V, torch.uint8)))


def oc_update_noalloc(x, dc, dv, mask, move, eta, target, oc_tol, xnew, result=None, stream=None):
    """topo_oc_update_noalloc: the OC update without a context or any allocation
    (device tensors: x, dc, dv, xnew FP64 and mask int8 of nel entries; result,
    if given, 3 FP64 entries receiving max |x_new - x|, the volume and lambda)."""
    import torch
    lib = load()
    nel = x.numel()
    _check(lib.topo_oc_update_noalloc(
        nel, _ptr(x, nel, torch.float64), _ptr(dc, nel, torch.float64), _ptr(dv, nel, torch.float64),
        _ptr(mask, nel, torch.int8), move, eta, target, oc_tol,
        None if stream is None else C.c_void_p(int(stream)), _ptr(xnew, nel, torch.float64),
        _ptr(result, 3, torch.float64)))


def _origin(origin):
    return None if origin is None else (C.c_double * 3)(*[float(v) for v in origin])


def surface_stl(dims, xphys, threshold=0.5, origin=None, h=1.0, stream=None):
    """topo_surface_stl: the binary STL image (a uint8 device tensor) of the
    thresholded design's voxel surface, and its triangle count."""
    import torch
    lib = load()
    nx, ny, nz = (int(v) for v in dims)
    nel = nx * ny * nz
    st = None if stream is None else C.c_void_p(int(stream))
    ntri = C.c_int64()
    _check(lib.topo_surface_stl(nx, ny, nz, _ptr(xphys, nel, torch.float64), threshold, _origin(origin), h, st,
                                None, 0, C.byref(ntri)))
    buf = torch.empty(84 + 50 * ntri.value, dtype=torch.uint8, device=xphys.device)
    _check(lib.topo_surface_stl(nx, ny, nz, _ptr(xphys, nel, torch.float64), threshold, _origin(origin), h, st,
                                _ptr(buf), buf.numel(), C.byref(ntri)))
    return buf, ntri.value


def write_stl(path, dims, xphys, threshold=0.5, origin=None, h=1.0):
    """Writes the binary STL of the thresholded design to a file (the image is
    built on the device by topo_surface_stl)."""
    buf, n = surface_stl(dims, xphys, threshold, origin, h)
    with open(path, "wb") as fh:
        fh.write(buf.cpu().numpy().tobytes())
    return n


def read_stl(path):
    """Triangles (n, 3, 3) float32 of a binary STL file (file parsing only)."""
    raw = open(path, "rb").read()
    if len(raw) < 84:
        raise ValueError("not a binary STL file")
    n = int(np.frombuffer(raw, dtype="<u4", count=1, offset=80)[0])
    if len(raw) < 84 + 50 * n:
        raise ValueError("truncated binary STL file")
    rec = np.dtype([("normal", "<f4", 3), ("v", "<f4", (3, 3)), ("attr", "<u2")])
    return np.ascontiguousarray(np.frombuffer(raw, dtype=rec, count=n, offset=84)["v"])


def voxelize(tri, dims, origin=None, h=1.0, code_inside=0, code_outside=1, stream=None):
    """topo_voxelize: int8 device mask of the elements whose centroid lies inside
    the closed mesh `tri` ((n, 3, 3) float32, host or device), and the number of
    element columns that saw an open mesh."""
    import torch
    lib = load()
    nx, ny, nz = (int(v) for v in dims)
    t = torch.as_tensor(np.ascontiguousarray(tri, dtype=np.float32)) if not isinstance(tri, torch.Tensor) else tri
    t = t.to("cuda").contiguous()
    mask = torch.empty(nx * ny * nz, dtype=torch.int8, device="cuda")
    bad = C.c_int64()
    ntri = t.numel() // 9
    _check(lib.topo_voxelize(_ptr(t, 9 * ntri, torch.float32) if ntri else None, ntri, nx, ny, nz,
                             _origin(origin), h, code_inside, code_outside,
                             None if stream is None else C.c_void_p(int(stream)), _ptr(mask), C.byref(bad)))
    return mask, bad.value


def default_train_opts(**kw) -> TrainOpts_C:
    lib = load()
    o = TrainOpts_C()
    lib.topo_default_train_opts(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(f"unknown training option {k}")
        setattr(o, k, v)
    return o


class Network:
    """The convolutional preconditioner network; wraps a topo_nn."""

    def __init__(self, channels=(16, 32, 64), stream=None, precision=PREC_FP32):
        lib = load()
        self._lib = lib
        import torch
        torch.cuda.init()
        ch = (C.c_int32 * 3)(*channels)
        h = C.c_void_p()
        _check(lib.topo_nn_create(ch, None if stream is None else C.c_void_p(int(stream)), C.byref(h)))
        self._h = h
        self.channels = tuple(channels)
        n = C.c_int64()
        _check(lib.topo_nn_n_params(self._h, C.byref(n)))
        self.n_params = n.value
        self.set_precision(precision)

    def set_precision(self, precision):
        _check(self._lib.topo_nn_set_precision(self._h, precision))
        self.precision = precision

    def close(self):
        if getattr(self, "_h", None):
            self._lib.topo_nn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_weights(self, blob):
        w = np.ascontiguousarray(blob, dtype=np.float32)
        if w.size != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters, got {w.size}")
        _check(self._lib.topo_nn_set_weights(self._h, w.ctypes.data_as(C.POINTER(C.c_float)), w.size))

    def get_weights(self) -> np.ndarray:
        w = np.empty(self.n_params, dtype=np.float32)
        _check(self._lib.topo_nn_get_weights(self._h, w.ctypes.data_as(C.POINTER(C.c_float)), w.size))
        return w

    @staticmethod
    def _nodes(nodes):
        return (C.c_int32 * 3)(*[int(v) for v in nodes])

    def forward(self, nodes, batch, x, out):
        """out[3][batch][V] = net(x[4][batch][V]); nodes = (NX, NY, NZ)."""
        import torch
        V = int(np.prod(nodes))
        _check(self._lib.topo_nn_forward(self._h, self._nodes(nodes), batch, _ptr(x, 4 * batch * V, torch.float32),
                                         _ptr(out, 3 * batch * V, torch.float32)))

    def loss_grad(self, nodes, rho, r, e, fixed, index, grad=None, loss=LOSS_REL) -> float:
        import torch
        V = int(np.prod(nodes))
        n = rho.numel() // V
        idx = np.ascontiguousarray(index, dtype=np.int32)
        value = C.c_double()
        _check(self._lib.topo_nn_loss_grad(
            self._h, self._nodes(nodes), n, _ptr(rho, n * V, torch.float32), _ptr(r, n * 3 * V, torch.float32),
            _ptr(e, n * 3 * V, torch.float32), _ptr(fixed, n * V, torch.uint8), idx.size,
            idx.ctypes.data_as(C.POINTER(C.c_int32)), loss, C.byref(value),
            _ptr(grad, self.n_params, torch.float32)))
        return value.value

    def train(self, nodes, rho, r, e, fixed, opts: Optional[TrainOpts_C] = None):
        import torch
        V = int(np.prod(nodes))
        n = rho.numel() // V
        o = opts if opts is not None else default_train_opts()
        ep = (C.c_double * max(1, o.epochs))()
        st = TrainStats_C()
        _check(self._lib.topo_nn_train(
            self._h, self._nodes(nodes), n, _ptr(rho, n * V, torch.float32), _ptr(r, n * 3 * V, torch.float32),
            _ptr(e, n * 3 * V, torch.float32), _ptr(fixed, n * V, torch.uint8), C.byref(o), ep, C.byref(st)))
        return {"steps": st.steps, "loss_first": st.loss_first, "loss_last": st.loss_last, "ms": st.ms,
                "epoch_loss": [ep[i] for i in range(o.epochs)]}


class Batch:
    """Independent problems iterated concurrently; wraps a topo_batch."""

    def __init__(self, problems, opts: Optional[Opts_C] = None, n_threads: int = 0):
        lib = load()
        self._lib = lib
        import torch
        torch.cuda.init()
        pcs, keep = [], []
        for p in problems:
            pc, k = _problem_c(p)
            pcs.append(pc)
            keep.append(k)
        arr = (Problem_C * len(pcs))(*pcs)
        self.opts = opts if opts is not None else default_opts()
        h = C.c_void_p()
        _check(lib.topo_setup_batch(arr, len(pcs), C.byref(self.opts), n_threads, C.byref(h)))
        self._h = h
        self.n = len(pcs)
        self.nel = [int(p.nelx * p.nely * p.nelz) for p in problems]
        self.ndof = [int(3 * (p.nelx + 1) * (p.nely + 1) * (p.nelz + 1)) for p in problems]

    def close(self):
        if getattr(self, "_h", None):
            self._lib.topo_destroy_batch(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def iterate(self, xs, n_iter: int, raise_on_nonconv=True) -> List[List[dict]]:
        import torch
        if len(xs) != self.n:
            raise ValueError("one design per problem")
        ptrs = (C.c_void_p * self.n)(*[_ptr(x, self.nel[i], torch.float64) for i, x in enumerate(xs)])
        stats = (IterStats_C * max(1, self.n * n_iter))()
        status = self._lib.topo_iterate_batch(self._h, ptrs, n_iter, stats)
        if not (status == TOPO_ENOTCONVERGED and not raise_on_nonconv):
            _check(status)
        return [[_iter_stats(stats[i * n_iter + k]) for k in range(n_iter)] for i in range(self.n)]

    def get_state(self, i: int, u=None, xphys=None):
        import torch
        c = C.c_void_p()
        _check(self._lib.topo_batch_context(self._h, i, C.byref(c)))
        _check(self._lib.topo_get_state(c, _ptr(u, self.ndof[i], torch.float64),
                                        _ptr(xphys, self.nel[i], torch.float64)))
