"""ctypes binding of libpsatd.so (argument marshalling only).

Every step of the PSATD path runs in the HIP library; this module converts
Python arguments into the C structs of ``include/psatd.h``, passes device
pointers and the current HIP stream, and turns status codes into exceptions.
PyTorch is used only to read tensor pointers, dtypes and the stream.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

_PKG = os.path.dirname(os.path.abspath(__file__))
LIBRARY_PATH = os.path.join(_PKG, "libpsatd.so")

PSATD_OK = 0
STATUS_NAMES = {
    0: "PSATD_OK", -1: "PSATD_ERR_INVALID_ARG", -2: "PSATD_ERR_UNSUPPORTED_SIZE",
    -3: "PSATD_ERR_OOM", -4: "PSATD_ERR_HIP", -5: "PSATD_ERR_WORKSPACE", -6: "PSATD_ERR_STATE",
}
PRECISION = {"fp32": 0, "fp64": 1}
SOURCE_MODE = {"vacuum": 0, "rho": 1, "j": 2}
PATH = {"fused": 0, "plain": 1}
FLAG_AUTOTUNE = 0x1
FLAG_GRAPH = 0x2
FLAG_NO_WORKSPACE = 0x4
FLAG_GENERIC_KERNELS = 0x8
FLAG_CENTERED_STENCIL = 0x10
FLAG_PSTD = 0x20
FLAG_RADIX4_LINES = 0x40
FDTD_SCHEME = {"yee": 0, "ckc": 1}

EXPORTED_SYMBOLS = (
    "psatd_plan", "psatd_workspace_size", "psatd_set_workspace", "psatd_push",
    "psatd_push_profiled", "psatd_pass_count", "psatd_pass_name", "psatd_pass_bytes",
    "psatd_plan_info", "psatd_destroy", "psatd_status_string", "psatd_last_error",
    "psatd_domain_create", "psatd_domain_local_shape", "psatd_domain_push", "psatd_domain_destroy",
    "psatd_fdtd_plan", "psatd_fdtd_push", "psatd_fdtd_destroy", "psatd_push_scratch",
    "psatd_plan_describe", "psatd_plan_tuning", "psatd_plan_tuned",
)
SCRATCH_BYTES = 256 << 20  # PSATD_SCRATCH_BYTES


class PatchDesc(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("reserved0", ctypes.c_int32),
                ("n", ctypes.c_int64 * 3), ("d", ctypes.c_double * 3),
                ("dt", ctypes.c_double), ("offset", ctypes.c_int64)]


class Config(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("source_mode", ctypes.c_int32),
                ("path", ctypes.c_int32), ("order", ctypes.c_int32),
                ("c", ctypes.c_double), ("eps0", ctypes.c_double),
                ("flags", ctypes.c_uint32), ("reserved0", ctypes.c_int32)]


class Fields(ctypes.Structure):
    _fields_ = [("E", ctypes.c_void_p * 3), ("B", ctypes.c_void_p * 3),
                ("J", ctypes.c_void_p * 3), ("rho_old", ctypes.c_void_p),
                ("rho_new", ctypes.c_void_p)]


class DomainDesc(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("reserved0", ctypes.c_int32),
                ("n", ctypes.c_int64 * 3), ("parts", ctypes.c_int32 * 3),
                ("guard", ctypes.c_int32 * 3), ("d", ctypes.c_double * 3),
                ("dt", ctypes.c_double)]


class PsatdError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None


def load_library(path: Optional[str] = None):
    """Load libpsatd.so (built in-tree); raises if it has not been built."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIBRARY_PATH
    if not os.path.exists(p):
        raise RuntimeError(
            f"{p} not found: the HIP library is not built (run `python -m "
            "paper_1608_05739_amd.build` or __graft_entry__.build()); there is no fallback")
    # torch ships its own HIP runtime.  Loading it before the library keeps
    # the process on the runtime torch uses: with the library's runtime loaded
    # and initialized first, torch's later initialization finds no GPU.
    import torch  # noqa: F401  (loaded for its HIP runtime; no device is touched)
    lib = ctypes.CDLL(p)
    vp, i32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
    lib.psatd_plan.argtypes = [ctypes.POINTER(Config), ctypes.POINTER(PatchDesc), i32, i32,
                               ctypes.POINTER(vp)]
    lib.psatd_plan_describe.argtypes = [ctypes.POINTER(Config), ctypes.POINTER(PatchDesc), i32,
                                        ctypes.POINTER(sz), ctypes.c_char_p, sz]
    lib.psatd_plan_tuned.argtypes = [ctypes.POINTER(Config), ctypes.POINTER(PatchDesc), i32, i32,
                                     ctypes.c_char_p, ctypes.POINTER(vp)]
    lib.psatd_plan_tuning.argtypes = [vp, ctypes.c_char_p, sz, ctypes.POINTER(sz)]
    lib.psatd_workspace_size.argtypes = [vp, ctypes.POINTER(sz)]
    lib.psatd_set_workspace.argtypes = [vp, vp, sz]
    lib.psatd_push.argtypes = [vp, ctypes.POINTER(Fields), i32, vp]
    lib.psatd_push_scratch.argtypes = [vp, ctypes.POINTER(Fields), i32, vp]
    lib.psatd_push_profiled.argtypes = [vp, ctypes.POINTER(Fields), i32, vp,
                                        ctypes.POINTER(ctypes.c_double), i32]
    lib.psatd_pass_count.argtypes = [vp, ctypes.POINTER(i32)]
    lib.psatd_pass_name.argtypes = [vp, i32]
    lib.psatd_pass_name.restype = ctypes.c_char_p
    lib.psatd_pass_bytes.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_double)]
    lib.psatd_plan_info.argtypes = [vp, ctypes.c_char_p, sz]
    lib.psatd_destroy.argtypes = [vp]
    lib.psatd_status_string.argtypes = [ctypes.c_int]
    lib.psatd_status_string.restype = ctypes.c_char_p
    lib.psatd_last_error.argtypes = []
    lib.psatd_last_error.restype = ctypes.c_char_p
    lib.psatd_domain_create.argtypes = [ctypes.POINTER(Config), ctypes.POINTER(DomainDesc), i32,
                                        ctypes.POINTER(vp)]
    lib.psatd_domain_local_shape.argtypes = [vp, ctypes.POINTER(ctypes.c_int64),
                                             ctypes.c_int64 * 3]
    lib.psatd_domain_push.argtypes = [vp, ctypes.POINTER(Fields), i32, vp]
    lib.psatd_domain_destroy.argtypes = [vp]
    lib.psatd_fdtd_plan.argtypes = [ctypes.POINTER(Config), i32, ctypes.POINTER(PatchDesc), i32,
                                    ctypes.POINTER(vp)]
    lib.psatd_fdtd_push.argtypes = [vp, ctypes.POINTER(Fields), i32, vp]
    lib.psatd_fdtd_destroy.argtypes = [vp]
    for name in ("psatd_plan", "psatd_plan_describe", "psatd_workspace_size", "psatd_set_workspace", "psatd_push",
                 "psatd_push_scratch", "psatd_push_profiled", "psatd_pass_count", "psatd_pass_bytes",
                 "psatd_plan_info", "psatd_destroy", "psatd_domain_create",
                 "psatd_domain_local_shape", "psatd_domain_push", "psatd_domain_destroy",
                 "psatd_fdtd_plan", "psatd_fdtd_push", "psatd_fdtd_destroy"):
        getattr(lib, name).restype = ctypes.c_int
    if path is None:
        _lib = lib
    return lib


def _check(lib, status: int):
    if status != PSATD_OK:
        raise PsatdError(status, lib.psatd_last_error().decode())


@dataclass
class Patch:
    """One periodic patch: n = (nx, ny, nz) (ny = 1 in 2D), d = (dx, dy, dz)."""

    ndim: int
    n: tuple
    d: tuple
    dt: float
    offset: Optional[int] = None

    @property
    def cells(self) -> int:
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])

    @property
    def shape(self):
        nx, ny, nz = self.n
        return (nz, nx) if self.ndim == 2 else (nz, ny, nx)


def as_patch(p) -> Patch:
    """Accept a Patch or any object with ndim, nx, ny, nz, dx, dy, dz, dt."""
    if isinstance(p, Patch):
        return p
    return Patch(int(p.ndim), (int(p.nx), int(p.ny), int(p.nz)),
                 (float(p.dx), float(p.dy), float(p.dz)), float(p.dt),
                 getattr(p, "offset", None))


def make_config(precision="fp32", source_mode="vacuum", path="fused", order=0, c=1.0, eps0=1.0,
                *, autotune=False, graph=False, allocate_workspace=True, generic_kernels=False,
                centered_stencil=False, pstd=False, radix4_lines=False) -> Config:
    cfg = Config()
    cfg.precision = PRECISION[precision]
    cfg.source_mode = SOURCE_MODE[source_mode]
    cfg.path = PATH[path]
    cfg.order = int(order)
    cfg.c = float(c)
    cfg.eps0 = float(eps0)
    cfg.flags = ((FLAG_AUTOTUNE if autotune else 0) | (FLAG_GRAPH if graph else 0)
                 | (0 if allocate_workspace else FLAG_NO_WORKSPACE)
                 | (FLAG_GENERIC_KERNELS if generic_kernels else 0)
                 | (FLAG_CENTERED_STENCIL if centered_stencil else 0)
                 | (FLAG_PSTD if pstd else 0)
                 | (FLAG_RADIX4_LINES if radix4_lines else 0))
    return cfg


def _field_struct(E, B, J, rho_old, rho_new, want_dtype, min_elements):
    import torch

    def ptr(t, name):
        if t is None:
            return None
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor")
        if not t.is_cuda:
            raise ValueError(f"{name} must be a device tensor")
        if t.dtype != want_dtype:
            raise TypeError(f"{name} has dtype {t.dtype}, expected {want_dtype}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if t.numel() < min_elements:
            raise ValueError(f"{name} holds {t.numel()} elements < {min_elements}")
        return t.data_ptr()

    f = Fields()
    for i in range(3):
        f.E[i] = ptr(E[i], f"E[{i}]")
        f.B[i] = ptr(B[i], f"B[{i}]")
        f.J[i] = ptr(J[i], f"J[{i}]") if J is not None else None
    f.rho_old = ptr(rho_old, "rho_old")
    f.rho_new = ptr(rho_new, "rho_new")
    return f


def _patch_descs(patches):
    """(patches, PatchDesc array, offsets, total elements); patches without an
    offset are packed in order, each padded to an even element count."""
    ps = [as_patch(p) for p in patches]
    off = 0
    offsets = []
    for p in ps:
        if p.offset is None:
            offsets.append(off)
            off += p.cells + (p.cells % 2)
        else:
            offsets.append(int(p.offset))
            off = max(off, int(p.offset) + p.cells)
    descs = (PatchDesc * max(1, len(ps)))()
    for i, p in enumerate(ps):
        descs[i].ndim = p.ndim
        descs[i].n = (ctypes.c_int64 * 3)(*[int(v) for v in p.n])
        descs[i].d = (ctypes.c_double * 3)(*[float(v) for v in p.d])
        descs[i].dt = float(p.dt)
        descs[i].offset = offsets[i]
    return ps, descs, offsets, off


def describe_plan(patches: Sequence, *, precision="fp32", source_mode="vacuum", path="fused",
                  order=0, c=1.0, eps0=1.0, generic_kernels=False, centered_stencil=False,
                  pstd=False, radix4_lines=False):
    """Plan on the host only (psatd_plan_describe): validates and lays out the
    plan without touching a device.  Returns (workspace bytes, pass
    description); raises PsatdError where Plan() would."""
    lib = load_library()
    ps, descs, _, _ = _patch_descs(patches)
    cfg = make_config(precision, source_mode, path, order, c, eps0,
                      generic_kernels=generic_kernels, centered_stencil=centered_stencil,
                      pstd=pstd, radix4_lines=radix4_lines)
    ws = ctypes.c_size_t()
    buf = ctypes.create_string_buffer(16384)
    _check(lib, lib.psatd_plan_describe(ctypes.byref(cfg), descs, len(ps), ctypes.byref(ws),
                                        buf, len(buf)))
    return ws.value, buf.value.decode()


class Plan:
    """A PSATD plan over one or more periodic patches on one HIP device.

    Component buffers are flat tensors holding every patch at its offset
    (by default the patches are packed in order, see :attr:`offsets`).
    ``pstd=True`` runs the PSTD contrast solver instead (leapfrog: B holds B
    at half-integer times; source_mode "vacuum" or "j").  ``radix4_lines=True``
    runs the generic line passes as radix-4 stages at 4 points per thread.
    ``tuning`` (a string from :attr:`tuning` of a plan with the same
    arguments) applies that plan's kernel choices instead of autotuning
    (``psatd_plan_tuned``).
    """

    def __init__(self, patches: Sequence, *, precision="fp32", source_mode="vacuum",
                 path="fused", order=0, c=1.0, eps0=1.0, autotune=False, graph=False,
                 device=0, allocate_workspace=True, generic_kernels=False,
                 centered_stencil=False, pstd=False, radix4_lines=False, tuning=None):
        self._lib = load_library()
        self._plan = None
        ps, descs, self.offsets, self.total_elements = _patch_descs(patches)
        self.patches = ps
        self.precision = precision
        self.source_mode = source_mode
        self.device = device
        cfg = make_config(precision, source_mode, path, order, c, eps0, autotune=autotune,
                          graph=graph, allocate_workspace=allocate_workspace,
                          generic_kernels=generic_kernels, centered_stencil=centered_stencil,
                          pstd=pstd, radix4_lines=radix4_lines)
        handle = ctypes.c_void_p()
        if tuning is None:
            _check(self._lib, self._lib.psatd_plan(ctypes.byref(cfg), descs, len(ps), int(device),
                                                    ctypes.byref(handle)))
        else:
            _check(self._lib, self._lib.psatd_plan_tuned(ctypes.byref(cfg), descs, len(ps),
                                                          int(device), tuning.encode(),
                                                          ctypes.byref(handle)))
        self._plan = handle

    # -------------------------------------------------------------- queries
    @property
    def tuning(self) -> str:
        """The plan's kernel choices (``psatd_plan_tuning``), for ``Plan(..., tuning=)``."""
        n = ctypes.c_size_t()
        _check(self._lib, self._lib.psatd_plan_tuning(self._plan, None, 0, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        _check(self._lib, self._lib.psatd_plan_tuning(self._plan, buf, n.value, None))
        return buf.value.decode()

    @property
    def workspace_size(self) -> int:
        n = ctypes.c_size_t()
        _check(self._lib, self._lib.psatd_workspace_size(self._plan, ctypes.byref(n)))
        return n.value

    @property
    def npass(self) -> int:
        n = ctypes.c_int32()
        _check(self._lib, self._lib.psatd_pass_count(self._plan, ctypes.byref(n)))
        return n.value

    @property
    def pass_names(self):
        return [self._lib.psatd_pass_name(self._plan, i).decode() for i in range(self.npass)]

    @property
    def pass_bytes(self):
        out = []
        for i in range(self.npass):
            b = ctypes.c_double()
            _check(self._lib, self._lib.psatd_pass_bytes(self._plan, i, ctypes.byref(b)))
            out.append(b.value)
        return out

    @property
    def info(self) -> str:
        buf = ctypes.create_string_buffer(8192)
        _check(self._lib, self._lib.psatd_plan_info(self._plan, buf, len(buf)))
        return buf.value.decode()

    def set_workspace(self, tensor):
        _check(self._lib, self._lib.psatd_set_workspace(
            self._plan, ctypes.c_void_p(tensor.data_ptr()),
            tensor.numel() * tensor.element_size()))
        self._ws_ref = tensor

    # -------------------------------------------------------------- push
    def _fields(self, E, B, J, rho_old, rho_new):
        import torch

        want = torch.float32 if self.precision == "fp32" else torch.float64
        return _field_struct(E, B, J, rho_old, rho_new, want, self.total_elements)

    @staticmethod
    def _stream(stream):
        import torch

        s = stream if stream is not None else torch.cuda.current_stream()
        return ctypes.c_void_p(s.cuda_stream)

    def push(self, E, B, J=None, rho_old=None, rho_new=None, steps=1, stream=None):
        """Advance E, B (lists of 3 tensors, updated in place) by ``steps`` steps."""
        f = self._fields(E, B, J, rho_old, rho_new)
        _check(self._lib, self._lib.psatd_push(self._plan, ctypes.byref(f), int(steps),
                                                self._stream(stream)))

    def push_scratch(self, E, B, J=None, rho_old=None, rho_new=None, steps=1, stream=None):
        """Like :meth:`push`, on the library's device-resident workspace
        (psatd_push_scratch: no allocation; workspace at most SCRATCH_BYTES)."""
        f = self._fields(E, B, J, rho_old, rho_new)
        _check(self._lib, self._lib.psatd_push_scratch(self._plan, ctypes.byref(f), int(steps),
                                                        self._stream(stream)))

    def push_profiled(self, E, B, J=None, rho_old=None, rho_new=None, steps=1, stream=None):
        """Like :meth:`push`; returns the mean milliseconds of each pass (HIP events)."""
        f = self._fields(E, B, J, rho_old, rho_new)
        n = self.npass
        ms = (ctypes.c_double * n)()
        _check(self._lib, self._lib.psatd_push_profiled(self._plan, ctypes.byref(f), int(steps),
                                                         self._stream(stream), ms, n))
        return list(ms)

    def close(self):
        if self._plan is not None:
            self._lib.psatd_destroy(self._plan)
            self._plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Domain:
    """Guard-cell domain decomposition of a periodic grid (Sec. II.A).

    ``n`` = (nx, ny, nz) global (ny = 1 in 2D), ``parts`` boxes per axis,
    ``guard`` cells per side on split axes.  :meth:`push` advances global E, B
    (flat tensors of nx*ny*nz elements) through the decomposed step.
    """

    def __init__(self, ndim, n, parts, guard, d, dt, *, precision="fp32", source_mode="vacuum",
                 path="fused", order=0, c=1.0, eps0=1.0, centered_stencil=False, graph=False,
                 autotune=False, device=0):
        self._lib = load_library()
        self._dom = None
        desc = DomainDesc()
        desc.ndim = int(ndim)
        desc.n = (ctypes.c_int64 * 3)(*[int(v) for v in n])
        desc.parts = (ctypes.c_int32 * 3)(*[int(v) for v in parts])
        desc.guard = (ctypes.c_int32 * 3)(*[int(v) for v in guard])
        desc.d = (ctypes.c_double * 3)(*[float(v) for v in d])
        desc.dt = float(dt)
        cfg = make_config(precision, source_mode, path, order, c, eps0, graph=graph,
                          autotune=autotune, centered_stencil=centered_stencil)
        handle = ctypes.c_void_p()
        _check(self._lib, self._lib.psatd_domain_create(ctypes.byref(cfg), ctypes.byref(desc),
                                                         int(device), ctypes.byref(handle)))
        self._dom = handle
        self.precision = precision
        self.cells = int(n[0]) * int(n[1]) * int(n[2])

    @property
    def local_shape(self):
        npatch = ctypes.c_int64()
        ln = (ctypes.c_int64 * 3)()
        _check(self._lib, self._lib.psatd_domain_local_shape(self._dom, ctypes.byref(npatch), ln))
        return npatch.value, tuple(ln)

    def push(self, E, B, J=None, rho_old=None, rho_new=None, steps=1, stream=None):
        import torch

        want = torch.float32 if self.precision == "fp32" else torch.float64
        f = _field_struct(E, B, J, rho_old, rho_new, want, self.cells)
        s = stream if stream is not None else torch.cuda.current_stream()
        _check(self._lib, self._lib.psatd_domain_push(self._dom, ctypes.byref(f), int(steps),
                                                       ctypes.c_void_p(s.cuda_stream)))

    def close(self):
        if self._dom is not None:
            self._lib.psatd_domain_destroy(self._dom)
            self._dom = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Fdtd:
    """FDTD contrast solver on one periodic patch (Sec. III.A, Table 1).

    ``scheme`` is "yee" (order 2, or order p) or "ckc" (2D, dx = dz).  Fields
    live on the staggered Yee grid, B at half-integer times; :meth:`push`
    advances flat tensors of nx*ny*nz elements (at ``offset``) in place.
    """

    def __init__(self, scheme, patch, *, precision="fp32", source_mode="vacuum", order=0, c=1.0,
                 eps0=1.0, offset=0, device=0):
        self._lib = load_library()
        self._h = None
        p = as_patch(patch)
        desc = PatchDesc()
        desc.ndim = p.ndim
        desc.n = (ctypes.c_int64 * 3)(*[int(v) for v in p.n])
        desc.d = (ctypes.c_double * 3)(*[float(v) for v in p.d])
        desc.dt = float(p.dt)
        desc.offset = int(offset if p.offset is None else p.offset)
        cfg = make_config(precision, source_mode, "fused", order, c, eps0)
        handle = ctypes.c_void_p()
        _check(self._lib, self._lib.psatd_fdtd_plan(ctypes.byref(cfg), FDTD_SCHEME[scheme],
                                                     ctypes.byref(desc), int(device),
                                                     ctypes.byref(handle)))
        self._h = handle
        self.precision = precision
        self.elements = int(desc.offset) + p.cells

    def push(self, E, B, J=None, steps=1, stream=None):
        import torch

        want = torch.float32 if self.precision == "fp32" else torch.float64
        f = _field_struct(E, B, J, None, None, want, self.elements)
        s = stream if stream is not None else torch.cuda.current_stream()
        _check(self._lib, self._lib.psatd_fdtd_push(self._h, ctypes.byref(f), int(steps),
                                                     ctypes.c_void_p(s.cuda_stream)))

    def close(self):
        if self._h is not None:
            self._lib.psatd_fdtd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
