"""Thin Python binding of the fftgal C ABI (``include/fftgal.h``).

Argument marshalling only: every step of the computation runs in the HIP
library ``_lib/libfftgal.so``.  PyTorch supplies the device workspace and the
stream.  There is no fallback: if the library is missing, loading raises.

The module-level functions carry the C names (``fftgal_plan``,
``fftgal_set_material``, ...); ``Plan`` is a small convenience wrapper that
owns a torch workspace tensor.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libfftgal.so")

FP64 = 0
FP32_ITER = 1
REDUCED_LEAN = 0x100  # reduced Ga laid out with one set of intermediates (shifts in turn)
TENSOR = 0x200  # d(d+1)/2 material fields per side (matrix images, anisotropic multi-phase inclusions)
CONCURRENT = 0x400  # per-solve buffers for all 2d solves: they may run at once
SEPARATE_PASSES = 0x800  # small 2D grids: per-pass kernels instead of one work-group per solve
FAST_GRID = 0x1000  # Ga plans: the double grid with specialised kernels if it holds at most 4x the points
PRECISIONS = {"fp64": FP64, "fp32": FP32_ITER, "fp32_iter": FP32_ITER}

STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ENOTCONV", -5: "ESTATE", -6: "EBREAKDOWN"}
EXPORTS = ("fftgal_workspace_bytes", "fftgal_workspace_bytes_p", "fftgal_plan", "fftgal_set_material",
           "fftgal_solve_primal", "fftgal_solve_dual", "fftgal_bounds", "fftgal_destroy",
           "fftgal_last_error", "fftgal_grid_size", "fftgal_set_timing", "fftgal_read_timing",
           "fftgal_warm_start", "fftgal_history", "fftgal_set_timing_classes", "fftgal_set_bound_tol",
           "fftgal_workspace_bytes_gani", "fftgal_plan_gani", "fftgal_bounds_of", "fftgal_envelope_images",
           "fftgal_workspace_bytes_reduced", "fftgal_plan_reduced", "fftgal_plan_static", "fftgal_solve_all",
           "fftgal_static_workspace_bytes",
           "fftgal_batch_workspace_bytes", "fftgal_batch_create", "fftgal_batch_add", "fftgal_batch_step",
           "fftgal_batch_poll", "fftgal_batch_destroy", "fftgal_batch_last_error")
KERNEL_CLASSES = ("expand", "pencil_inv", "row", "pencil_fwd", "project", "cg_update", "cg_scalar", "rhs",
                  "bounds", "setup", "checkpoint", "solo")


class FftgalError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (STATUS.get(code, "?"), code, msg))
        self.code = code


class Material(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32),
        ("A0", ctypes.c_double * 9),
        ("n_incl", ctypes.c_int32),
        ("shape", ctypes.POINTER(ctypes.c_int32)),
        ("center", ctypes.POINTER(ctypes.c_double)),
        ("size", ctypes.POINTER(ctypes.c_double)),
        ("A_in", ctypes.POINTER(ctypes.c_double)),
        ("P", ctypes.c_int32 * 3),
        ("image", ctypes.POINTER(ctypes.c_double)),
        ("image_device", ctypes.c_int32),
        ("image_dual", ctypes.POINTER(ctypes.c_double)),
        ("image_tensor", ctypes.c_int32),
    ]


class Info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("rel_res", ctypes.c_double), ("res0", ctypes.c_double),
                ("stagnated", ctypes.c_int32), ("iterate", ctypes.c_int32)]

    def as_dict(self):
        return {"iters": int(self.iters), "converged": bool(self.converged),
                "rel_res": float(self.rel_res), "res0": float(self.res0),
                "stagnated": bool(self.stagnated), "iterate": int(self.iterate)}


_LIB = None


def load_library(path=LIB_PATH):
    """Load libfftgal.so (after torch, so that both share one HIP runtime)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise FileNotFoundError(
            "libfftgal.so is not built (%s); run python -m paper_1412_2033_amd.build" % path)
    try:
        import torch  # noqa: F401  (load the HIP runtime torch uses first)
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    i32p = ctypes.POINTER(ctypes.c_int32)
    vp = ctypes.c_void_p
    lib.fftgal_workspace_bytes.argtypes = [ctypes.c_int, i32p, ctypes.c_int]
    lib.fftgal_workspace_bytes.restype = ctypes.c_size_t
    lib.fftgal_workspace_bytes_p.argtypes = [ctypes.c_int, i32p, ctypes.c_int, i32p]
    lib.fftgal_workspace_bytes_p.restype = ctypes.c_size_t
    lib.fftgal_plan.argtypes = [ctypes.POINTER(vp), ctypes.c_int, i32p, ctypes.c_int, vp, ctypes.c_size_t, vp]
    lib.fftgal_plan.restype = ctypes.c_int
    lib.fftgal_set_material.argtypes = [vp, ctypes.POINTER(Material)]
    lib.fftgal_set_material.restype = ctypes.c_int
    lib.fftgal_solve_all.argtypes = [vp, ctypes.c_double, ctypes.c_int, ctypes.POINTER(Info)]
    lib.fftgal_solve_all.restype = ctypes.c_int
    for name in ("fftgal_solve_primal", "fftgal_solve_dual"):
        f = getattr(lib, name)
        f.argtypes = [vp, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.POINTER(Info)]
        f.restype = ctypes.c_int
    dp = ctypes.POINTER(ctypes.c_double)
    lib.fftgal_bounds.argtypes = [vp, dp, dp, dp]
    lib.fftgal_bounds.restype = ctypes.c_int
    lib.fftgal_destroy.argtypes = [vp]
    lib.fftgal_destroy.restype = ctypes.c_int
    lib.fftgal_last_error.argtypes = [vp]
    lib.fftgal_last_error.restype = ctypes.c_char_p
    lib.fftgal_grid_size.argtypes = [vp, ctypes.c_int]
    lib.fftgal_grid_size.restype = ctypes.c_int
    lib.fftgal_set_timing.argtypes = [vp, ctypes.c_int]
    lib.fftgal_set_timing.restype = ctypes.c_int
    lib.fftgal_read_timing.argtypes = [vp, ctypes.POINTER(ctypes.c_double), i32p]
    lib.fftgal_read_timing.restype = ctypes.c_int
    lib.fftgal_set_timing_classes.argtypes = [vp, ctypes.c_uint32]
    lib.fftgal_set_timing_classes.restype = ctypes.c_int
    lib.fftgal_set_bound_tol.argtypes = [vp, ctypes.c_double]
    lib.fftgal_set_bound_tol.restype = ctypes.c_int
    lib.fftgal_workspace_bytes_gani.argtypes = [ctypes.c_int, i32p, ctypes.c_int, i32p]
    lib.fftgal_workspace_bytes_gani.restype = ctypes.c_size_t
    lib.fftgal_plan_static.argtypes = [ctypes.POINTER(vp), ctypes.c_int, i32p, ctypes.c_int, vp]
    lib.fftgal_plan_static.restype = ctypes.c_int
    lib.fftgal_static_workspace_bytes.argtypes = []
    lib.fftgal_static_workspace_bytes.restype = ctypes.c_size_t
    lib.fftgal_plan_gani.argtypes = [ctypes.POINTER(vp), ctypes.c_int, i32p, ctypes.c_int, vp, ctypes.c_size_t, vp]
    lib.fftgal_plan_gani.restype = ctypes.c_int
    lib.fftgal_workspace_bytes_reduced.argtypes = [ctypes.c_int, i32p, ctypes.c_int, i32p]
    lib.fftgal_workspace_bytes_reduced.restype = ctypes.c_size_t
    lib.fftgal_plan_reduced.argtypes = [ctypes.POINTER(vp), ctypes.c_int, i32p, ctypes.c_int, vp, ctypes.c_size_t,
                                        vp]
    lib.fftgal_plan_reduced.restype = ctypes.c_int
    lib.fftgal_bounds_of.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double)]
    lib.fftgal_bounds_of.restype = ctypes.c_int
    lib.fftgal_envelope_images.argtypes = [vp, ctypes.POINTER(Material), i32p, vp, vp]
    lib.fftgal_envelope_images.restype = ctypes.c_int
    lib.fftgal_warm_start.argtypes = [vp, vp]
    lib.fftgal_warm_start.restype = ctypes.c_int
    lib.fftgal_history.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.c_int,
                                   i32p]
    lib.fftgal_history.restype = ctypes.c_int
    lib.fftgal_batch_workspace_bytes.argtypes = [ctypes.c_int]
    lib.fftgal_batch_workspace_bytes.restype = ctypes.c_size_t
    lib.fftgal_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, vp, ctypes.c_size_t, vp]
    lib.fftgal_batch_create.restype = ctypes.c_int
    lib.fftgal_batch_add.argtypes = [vp, vp, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int, i32p]
    lib.fftgal_batch_add.restype = ctypes.c_int
    lib.fftgal_batch_step.argtypes = [vp, ctypes.c_int, i32p]
    lib.fftgal_batch_step.restype = ctypes.c_int
    lib.fftgal_batch_poll.argtypes = [vp, i32p, ctypes.POINTER(Info), i32p]
    lib.fftgal_batch_poll.restype = ctypes.c_int
    lib.fftgal_batch_destroy.argtypes = [vp]
    lib.fftgal_batch_destroy.restype = ctypes.c_int
    lib.fftgal_batch_last_error.argtypes = [vp]
    lib.fftgal_batch_last_error.restype = ctypes.c_char_p
    _LIB = lib
    return lib


def _i32(vals):
    arr = (ctypes.c_int32 * 3)()
    for i, v in enumerate(vals):
        arr[i] = int(v)
    return arr


def _check(code, plan=None):
    if code != 0:
        msg = load_library().fftgal_last_error(plan).decode()
        raise FftgalError(code, msg)


# ---- C-named functions (marshalling only) ------------------------------------

def fftgal_workspace_bytes(d, N, precision=FP64, P=None, scheme="ga"):
    lib = load_library()
    if scheme == "gani":
        return int(lib.fftgal_workspace_bytes_gani(d, _i32(N), precision, None if P is None else _i32(P)))
    if scheme == "reduced":
        return int(lib.fftgal_workspace_bytes_reduced(d, _i32(N), precision, None if P is None else _i32(P)))
    if P is None:
        return int(lib.fftgal_workspace_bytes(d, _i32(N), precision))
    return int(lib.fftgal_workspace_bytes_p(d, _i32(N), precision, _i32(P)))


def fftgal_plan(d, N, precision, workspace_ptr, nbytes, stream_ptr, scheme="ga"):
    lib = load_library()
    h = ctypes.c_void_p()
    fn = {"gani": lib.fftgal_plan_gani, "reduced": lib.fftgal_plan_reduced}.get(scheme, lib.fftgal_plan)
    _check(fn(ctypes.byref(h), d, _i32(N), precision, ctypes.c_void_p(workspace_ptr), nbytes,
              ctypes.c_void_p(stream_ptr)), None)
    return h


def fftgal_plan_static(d, N, precision, stream_ptr):
    """A plan on the library's static device workspace (no device allocation)."""
    h = ctypes.c_void_p()
    _check(load_library().fftgal_plan_static(ctypes.byref(h), d, _i32(N), precision, ctypes.c_void_p(stream_ptr)),
           None)
    return h


def fftgal_static_workspace_bytes():
    return int(load_library().fftgal_static_workspace_bytes())


def fftgal_bounds_of(plan, src, d):
    up = (ctypes.c_double * (d * d))()
    lo = (ctypes.c_double * (d * d))()
    gap = ctypes.c_double()
    _check(load_library().fftgal_bounds_of(plan, src, up, lo, ctypes.byref(gap)), plan)
    return (np.array(up[:]).reshape(d, d), np.array(lo[:]).reshape(d, d), float(gap.value))


def material_struct(micro):
    """Marshal a ``synth`` microstructure dict into an fftgal_material (keeps arrays alive)."""
    d = int(micro["d"])
    m = Material()
    keep = []
    if micro["kind"] == "inclusions":
        m.kind = 0
        A0 = np.asarray(micro["A0"], float).reshape(d, d)
        for i in range(d * d):
            m.A0[i] = A0.ravel()[i]
        shapes = np.array([0 if s == "rect" else 1 if s == "circ" else -1 for s in micro["shapes"]], np.int32)
        centers = np.ascontiguousarray(micro["centers"], float).reshape(-1)
        sizes = np.ascontiguousarray(micro["sizes"], float).reshape(-1)
        ain = np.ascontiguousarray(micro["A_in"], float).reshape(-1)
        keep += [shapes, centers, sizes, ain]
        m.n_incl = len(shapes)
        m.shape = shapes.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        m.center = centers.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        m.size = sizes.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        m.A_in = ain.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    elif micro["kind"] == "voxels":
        m.kind = 1
        for a in range(d):
            m.P[a] = int(micro["P"][a])
        img = micro["image"]
        dual = micro.get("image_dual")
        on_device = hasattr(img, "data_ptr") and getattr(img, "is_cuda", False)
        if dual is not None and (hasattr(dual, "data_ptr") and getattr(dual, "is_cuda", False)) != on_device:
            raise ValueError("image and image_dual must both be host arrays or both device tensors")

        def ptr(a):
            if on_device:
                # a torch float64 tensor already resident on the device
                if not a.is_contiguous() or str(a.dtype) != "torch.float64":
                    raise ValueError("device image must be a contiguous float64 tensor")
                keep.append(a)
                return ctypes.cast(ctypes.c_void_p(a.data_ptr()), ctypes.POINTER(ctypes.c_double))
            a = np.ascontiguousarray(a, float)
            keep.append(a)
            return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))

        m.image = ptr(img)
        m.image_device = 1 if on_device else 0
        # a matrix per voxel: shape P + (d, d)
        m.image_tensor = 1 if len(tuple(img.shape)) == d + 2 else 0
        if dual is not None:
            m.image_dual = ptr(dual)
    else:
        raise ValueError(micro["kind"])
    return m, keep


def fftgal_set_material(plan, micro):
    m, keep = material_struct(micro)
    _check(load_library().fftgal_set_material(plan, ctypes.byref(m)), plan)
    del keep


def _solve(fn, plan, d, alpha, rtol, maxit):
    n = d if alpha < 0 else 1
    infos = (Info * n)()
    code = fn(plan, alpha, rtol, maxit, infos)
    if code not in (0, -4):
        _check(code, plan)
    return [i.as_dict() for i in infos], code


def fftgal_solve_primal(plan, d, alpha=-1, rtol=1e-10, maxit=20000):
    return _solve(load_library().fftgal_solve_primal, plan, d, alpha, rtol, maxit)


def fftgal_solve_dual(plan, d, alpha=-1, rtol=1e-10, maxit=20000):
    return _solve(load_library().fftgal_solve_dual, plan, d, alpha, rtol, maxit)


def fftgal_solve_all(plan, d, rtol=1e-10, maxit=20000):
    """All 2d solves: ([primal infos], [dual infos], status code)."""
    infos = (Info * (2 * d))()
    code = load_library().fftgal_solve_all(plan, rtol, maxit, infos)
    if code not in (0, -4):
        _check(code, plan)
    out = [i.as_dict() for i in infos]
    return out[:d], out[d:], code


def fftgal_bounds(plan, d):
    up = (ctypes.c_double * (d * d))()
    lo = (ctypes.c_double * (d * d))()
    gap = ctypes.c_double()
    _check(load_library().fftgal_bounds(plan, up, lo, ctypes.byref(gap)), plan)
    return (np.array(up[:]).reshape(d, d), np.array(lo[:]).reshape(d, d), float(gap.value))


def fftgal_destroy(plan):
    return load_library().fftgal_destroy(plan)


def fftgal_last_error(plan=None):
    return load_library().fftgal_last_error(plan).decode()


def fftgal_grid_size(plan, axis):
    return int(load_library().fftgal_grid_size(plan, axis))


def fftgal_set_timing(plan, enable):
    _check(load_library().fftgal_set_timing(plan, int(bool(enable))), plan)


def fftgal_set_timing_classes(plan, classes):
    mask = 0
    for c in classes:
        mask |= 1 << KERNEL_CLASSES.index(c)
    _check(load_library().fftgal_set_timing_classes(plan, mask), plan)


def fftgal_set_bound_tol(plan, btol):
    _check(load_library().fftgal_set_bound_tol(plan, float(btol)), plan)


def fftgal_read_timing(plan):
    """{class: (milliseconds, launches)} since the previous read."""
    n = len(KERNEL_CLASSES)
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_int32 * n)()
    _check(load_library().fftgal_read_timing(plan, ms, cnt), plan)
    return {c: (float(ms[i]), int(cnt[i])) for i, c in enumerate(KERNEL_CLASSES)}


def fftgal_warm_start(fine, coarse):
    _check(load_library().fftgal_warm_start(fine, coarse), fine)


def fftgal_history(plan, kind, alpha, cap=20001):
    """Energies of the CG iterates of the last (kind 0 primal / 1 dual, alpha) solve."""
    buf = (ctypes.c_double * cap)()
    n = ctypes.c_int32()
    _check(load_library().fftgal_history(plan, int(kind), int(alpha), buf, int(cap), ctypes.byref(n)), plan)
    return np.array(buf[:min(cap, n.value)])


# ---- convenience wrapper ------------------------------------------------------

class Plan:
    """A plan plus the torch device workspace it runs in."""

    def __init__(self, d, N, precision="fp64", device="cuda", stream=None, P=None, scheme="ga", lean=False,
                 tensor=False, concurrent=False, separate_passes=False, fast_grid=False):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("fftgal needs a HIP device")
        self.d = int(d)
        self.N = tuple(int(n) for n in N)
        self.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        self.scheme = scheme
        flags = self.precision | (REDUCED_LEAN if lean else 0) | (TENSOR if tensor else 0) | \
            (CONCURRENT if concurrent else 0) | (SEPARATE_PASSES if separate_passes else 0) | \
            (FAST_GRID if fast_grid else 0)
        self.concurrent = bool(concurrent)
        self.nbytes = fftgal_workspace_bytes(self.d, self.N, flags, P, scheme)
        if self.nbytes == 0:
            raise FftgalError(-1, "invalid plan arguments")
        dev = torch.device(device)
        self.workspace = torch.empty(self.nbytes, dtype=torch.uint8, device=dev)
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        self.handle = fftgal_plan(self.d, self.N, flags, self.workspace.data_ptr(), self.nbytes,
                                  self.stream.cuda_stream, scheme)
        self.M = tuple(fftgal_grid_size(self.handle, a) for a in range(self.d))

    def set_material(self, micro):
        fftgal_set_material(self.handle, micro)

    def solve_primal(self, alpha=-1, rtol=1e-10, maxit=20000):
        return fftgal_solve_primal(self.handle, self.d, alpha, rtol, maxit)

    def solve_dual(self, alpha=-1, rtol=1e-10, maxit=20000):
        return fftgal_solve_dual(self.handle, self.d, alpha, rtol, maxit)

    def bounds(self):
        return fftgal_bounds(self.handle, self.d)

    def set_timing(self, enable=True, classes=None):
        """Time every launch (enable), or only the given kernel classes."""
        if classes is None:
            fftgal_set_timing(self.handle, enable)
        else:
            fftgal_set_timing_classes(self.handle, classes if enable else ())

    def set_bound_tol(self, btol):
        fftgal_set_bound_tol(self.handle, btol)

    def read_timing(self):
        return fftgal_read_timing(self.handle)

    def envelope_images(self, micro, P):
        """Upper and lower voxel images (device float64 tensors of shape P) of an
        inclusion description, for upper-upper / lower-lower bounds."""
        import torch
        P = tuple(int(p) for p in P)
        up = torch.empty(P, dtype=torch.float64, device=self.workspace.device)
        lo = torch.empty(P, dtype=torch.float64, device=self.workspace.device)
        m, keep = material_struct(micro)
        _check(load_library().fftgal_envelope_images(self.handle, ctypes.byref(m), _i32(P), up.data_ptr(),
                                                     lo.data_ptr()), self.handle)
        del keep
        return up, lo

    def bounds_of(self, src):
        """Guaranteed bounds from the fields of the solved Plan `src` (e.g. GaNi)."""
        return fftgal_bounds_of(self.handle, src.handle, self.d)

    def warm_start(self, coarse):
        """Start the next solves from the finished solves of `coarse` (a Plan)."""
        fftgal_warm_start(self.handle, coarse.handle)

    def history(self, kind, alpha):
        return fftgal_history(self.handle, kind, alpha)

    def run(self, micro, rtol=1e-10, maxit=20000, warm_from=None):
        """set_material (+ warm start from the solved Plan `warm_from`) + all 2d
        solves + bounds; returns a result dict."""
        self.set_material(micro)
        if warm_from is not None:
            self.warm_start(warm_from)
        if self.concurrent:
            ip, idl, code = fftgal_solve_all(self.handle, self.d, rtol, maxit)
            cp = cd = code
        else:
            ip, cp = self.solve_primal(-1, rtol, maxit)
            idl, cd = self.solve_dual(-1, rtol, maxit)
        up, lo, gap = self.bounds()
        return {"upper": up, "lower": lo, "gap": gap, "info_primal": ip, "info_dual": idl,
                "status_primal": cp, "status_dual": cd}

    def close(self):
        if getattr(self, "handle", None) is not None:
            fftgal_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- batched CG (continuous batching) --------------------------------------------

def _bcheck(code, batch):
    if code != 0:
        raise FftgalError(code, load_library().fftgal_batch_last_error(batch).decode())


def fftgal_batch_workspace_bytes(capacity):
    return int(load_library().fftgal_batch_workspace_bytes(int(capacity)))


def fftgal_batch_create(capacity, workspace_ptr, nbytes, stream_ptr):
    h = ctypes.c_void_p()
    code = load_library().fftgal_batch_create(ctypes.byref(h), int(capacity), ctypes.c_void_p(workspace_ptr),
                                              nbytes, ctypes.c_void_p(stream_ptr))
    if code != 0:
        raise FftgalError(code, load_library().fftgal_last_error(None).decode())
    return h


def fftgal_batch_add(batch, plan, kind, alpha, rtol, maxit):
    sid = ctypes.c_int32()
    _bcheck(load_library().fftgal_batch_add(batch, plan, int(kind), int(alpha), float(rtol), int(maxit),
                                            ctypes.byref(sid)), batch)
    return int(sid.value)


def fftgal_batch_step(batch, iterations):
    n = ctypes.c_int32()
    _bcheck(load_library().fftgal_batch_step(batch, int(iterations), ctypes.byref(n)), batch)
    return int(n.value)


def fftgal_batch_poll(batch):
    """(solve_id, info dict, status code) of one retired solve, or None."""
    sid = ctypes.c_int32()
    info = Info()
    st = ctypes.c_int32()
    if load_library().fftgal_batch_poll(batch, ctypes.byref(sid), ctypes.byref(info), ctypes.byref(st)) == 0:
        return None
    return int(sid.value), info.as_dict(), int(st.value)


def fftgal_batch_destroy(batch):
    return load_library().fftgal_batch_destroy(batch)


class Batch:
    """A batch plus its torch device workspace; plans added must share its stream."""

    def __init__(self, capacity=256, device="cuda", stream=None):
        import torch
        dev = torch.device(device)
        self.capacity = int(capacity)
        self.nbytes = fftgal_batch_workspace_bytes(self.capacity)
        self.workspace = torch.empty(self.nbytes, dtype=torch.uint8, device=dev)
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        self.handle = fftgal_batch_create(self.capacity, self.workspace.data_ptr(), self.nbytes,
                                          self.stream.cuda_stream)

    def add(self, plan, kind, alpha, rtol=1e-10, maxit=20000):
        return fftgal_batch_add(self.handle, plan.handle, kind, alpha, rtol, maxit)

    def step(self, iterations=8):
        return fftgal_batch_step(self.handle, iterations)

    def poll(self):
        out = []
        while True:
            r = fftgal_batch_poll(self.handle)
            if r is None:
                return out
            out.append(r)

    def close(self):
        if getattr(self, "handle", None) is not None:
            fftgal_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

