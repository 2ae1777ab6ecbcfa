"""MI355X phase-field stepper: Python binding of libpfsolve.so.

Every step of the model runs in the HIP kernels behind the C ABI declared in
``include/pfsolve.h``; this module only marshals arguments.  PyTorch is used
for device memory (borrowed buffers) and streams.  There is no CPU fallback:
if the library is not built, loading fails with an error.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import numpy as np

from . import _capi as A

__all__ = ["PfError", "Domain", "Pack", "load", "set_variant", "required_bytes",
           "diag_fields_noalloc"]

_lib = None
_lock = threading.Lock()


class PfError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        super().__init__(f"{A.STATUS_NAMES.get(status, status)}: {message}")


def load() -> C.CDLL:
    """Load libpfsolve.so (torch first, so both share one HIP runtime)."""
    global _lib
    with _lock:
        if _lib is None:
            import torch  # noqa: F401  (binds the HIP runtime soname to torch's copy)

            if not os.path.exists(A.LIB_PATH):
                raise RuntimeError(
                    f"{A.LIB_PATH} is not built: run __graft_entry__.build() first")
            _lib = A.declare(C.CDLL(A.LIB_PATH))
    return _lib


def _check(status: int):
    if status != A.PF_OK:
        raise PfError(status, load().pf_last_error().decode())


def set_variant(variant: int):
    """0 = direct (six faces per cell), 1 = tiled (every face once)."""
    _check(load().pf_set_variant(int(variant)))


def _prec_code(prec) -> int:
    if prec in ("fp64", "f64", A.PF_FP64):
        return A.PF_FP64
    if prec in ("fp32", "f32", A.PF_FP32):
        return A.PF_FP32
    raise ValueError(f"unknown precision {prec!r}")


def required_bytes(shape, prec="fp64", dx: float = 1.0) -> int:
    nz, ny, nx = shape
    desc = A.PfDomainDesc(nx, ny, nz, _prec_code(prec), dx)
    out = C.c_size_t()
    _check(load().pf_required_bytes(C.byref(desc), C.byref(out)))
    return out.value


def _stream_handle(stream) -> int:
    if stream is None:
        return 0
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


def params_struct(p: dict) -> A.PfParams:
    s = A.PfParams()
    s.eps = p["eps"]
    s.gamma3 = p["gamma3"]
    for a in range(4):
        s.tau[a] = p["tau"][a]
        s.w0[a] = p["w0"][a]
        s.w1[a] = p["w1"][a]
        s.D[a] = p["D"][a]
        for b in range(4):
            s.gamma[a][b] = p["gamma"][a][b]
            s.aniso_delta[a][b] = p["delta"][a][b]
        for q in range(2):
            s.chi0[a][q] = p["chi0"][a][q]
            s.chi1[a][q] = p["chi1"][a][q]
            s.c0[a][q] = p["c0"][a][q]
            s.c1[a][q] = p["c1"][a][q]
    for k in ("TE", "T0", "G", "v", "zoff", "dt"):
        setattr(s, k, float(p[k]))
    s.antitrapping = int(p.get("antitrapping", 1))
    s.mu_frozen = int(p.get("mu_frozen", 0))
    s.diag_every = int(p.get("diag_every", 0))
    s.shortcuts = int(p.get("shortcuts", 1))
    s.window_z = int(p.get("window_z", 0))
    s.top_bc = int(p.get("top_bc", 0))
    fill = p.get("mu_fill", (0.0, 0.0))
    s.mu_fill[0], s.mu_fill[1] = float(fill[0]), float(fill[1])
    return s


def _diag_dict(dg) -> dict:
    return {
        "t": dg.t, "step": dg.step, "sum_c": list(dg.sum_c), "sum_phi": list(dg.sum_phi),
        "max_simplex_dev": dg.max_simplex_dev, "phi_min": dg.phi_min,
        "phi_max": dg.phi_max, "nonfinite": dg.nonfinite,
        "window_shifts": dg.window_shifts,
        "light_items": dg.light_items, "work_items": dg.work_items,
        "fixed_items": dg.fixed_items, "mu_pure_items": dg.mu_pure_items,
        "copied_items": dg.copied_items,
    }


def diag_fields_noalloc(fields, params: dict, t: float, dx: float = 1.0, stream=None,
                        raise_nonfinite: bool = True) -> dict:
    """Diagnostics of a torch CUDA tensor ``fields`` of shape (6, nz, ny, nx)
    (phi_0..3, mu_0, mu_1; float64 or float32, contiguous) at time t, by
    pf_diag_fields_noalloc: no domain, no device allocation."""
    import torch

    if fields.dim() != 4 or fields.shape[0] != 6 or not fields.is_contiguous():
        raise ValueError("fields must be a contiguous (6, nz, ny, nx) tensor")
    if fields.dtype == torch.float64:
        prec = A.PF_FP64
    elif fields.dtype == torch.float32:
        prec = A.PF_FP32
    else:
        raise ValueError("fields must be float64 or float32")
    _, nz, ny, nx = (int(v) for v in fields.shape)
    desc = A.PfDomainDesc(nx, ny, nz, prec, float(dx))
    ps = params_struct(params)
    dg = A.PfDiag()
    st = load().pf_diag_fields_noalloc(C.byref(desc), C.byref(ps), C.c_void_p(fields.data_ptr()),
                                       float(t), C.c_void_p(_stream_handle(stream)), C.byref(dg))
    if st != A.PF_OK and (raise_nonfinite or st != A.PF_ERR_NONFINITE):
        _check(st)
    return _diag_dict(dg)


class Domain:
    """One grid of nx*ny*nz cells with its fields resident on the GPU.

    shape = (nz, ny, nx).  ``buffer``: optional torch uint8 CUDA tensor lent
    to the library (it must stay alive while the domain exists).
    """

    def __init__(self, shape, prec="fp64", dx: float = 1.0, buffer=None, stream=None):
        lib = load()
        nz, ny, nx = (int(v) for v in shape)
        self.shape = (nz, ny, nx)
        self.prec = "fp64" if _prec_code(prec) == A.PF_FP64 else "fp32"
        self.dx = float(dx)
        self._buffer = buffer
        self.stream = stream
        desc = A.PfDomainDesc(nx, ny, nz, _prec_code(prec), float(dx))
        borrowed = None
        if buffer is not None:
            borrowed = A.PfDeviceBuffer(C.c_void_p(buffer.data_ptr()),
                                        buffer.numel() * buffer.element_size())
        h = C.c_void_p()
        _check(lib.pf_create_domain(C.byref(desc), C.byref(borrowed) if borrowed else None,
                                    C.c_void_p(_stream_handle(stream)), C.byref(h)))
        self._h = h

    # ------------------------------------------------------------ lifecycle
    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("domain is closed")
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None:
            load().pf_destroy(self._h)
            self._h = None
            self._buffer = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ------------------------------------------------------------ setup
    def set_params(self, p: dict):
        self.params = dict(p)
        _check(load().pf_set_params(self.handle, C.byref(params_struct(p))))

    @property
    def dt(self) -> float:
        dt, bound = C.c_double(), C.c_double()
        _check(load().pf_get_dt(self.handle, C.byref(dt), C.byref(bound)))
        return dt.value

    @property
    def bound(self) -> float:
        dt, bound = C.c_double(), C.c_double()
        _check(load().pf_get_dt(self.handle, C.byref(dt), C.byref(bound)))
        return bound.value

    def init_voronoi(self, seed: int, nseeds: int, solid_height: int, mu_init=(0.0, 0.0)):
        ini = A.PfInit()
        ini.kind = A.PF_INIT_VORONOI
        ini.seed = int(seed) & ((1 << 64) - 1)
        ini.nseeds = int(nseeds)
        ini.solid_height = int(solid_height)
        ini.mu_init[0], ini.mu_init[1] = float(mu_init[0]), float(mu_init[1])
        _check(load().pf_init_fields(self.handle, C.byref(ini)))

    def init_host(self, phi: np.ndarray, mu: np.ndarray):
        nz, ny, nx = self.shape
        phi = np.ascontiguousarray(phi, dtype=np.float64)
        mu = np.ascontiguousarray(mu, dtype=np.float64)
        if phi.shape != (4, nz, ny, nx) or mu.shape != (2, nz, ny, nx):
            raise ValueError("phi must be (4,nz,ny,nx) and mu (2,nz,ny,nx)")
        ini = A.PfInit()
        ini.kind = A.PF_INIT_HOST
        ini.phi = phi.ctypes.data_as(C.POINTER(C.c_double))
        ini.mu = mu.ctypes.data_as(C.POINTER(C.c_double))
        _check(load().pf_init_fields(self.handle, C.byref(ini)))

    def set_time(self, step: int):
        _check(load().pf_set_time(self.handle, int(step)))

    # ------------------------------------------------------------ stepping
    def step(self, n: int = 1):
        _check(load().pf_step(self.handle, int(n)))

    def step_timed(self, n: int = 1):
        """Run n steps; return (phi-sweep ms, mu-sweep ms) summed over them."""
        a, b = C.c_double(0.0), C.c_double(0.0)
        _check(load().pf_step_timed(self.handle, int(n), C.byref(a), C.byref(b)))
        return a.value, b.value

    def sync(self):
        _check(load().pf_sync(self.handle))

    @property
    def step_index(self) -> int:
        s = C.c_int64()
        _check(load().pf_get_step(self.handle, C.byref(s)))
        return s.value

    # ------------------------------------------------------------ readback
    def read(self):
        nz, ny, nx = self.shape
        phi = np.empty((4, nz, ny, nx))
        mu = np.empty((2, nz, ny, nx))
        _check(load().pf_read_fields(self.handle, phi.ctypes.data_as(C.POINTER(C.c_double)),
                                     mu.ctypes.data_as(C.POINTER(C.c_double)), None))
        return phi, mu

    # ------------------------------------------------------------ output
    def save_checkpoint(self, path: str):
        """FP32 checkpoint of the current state (format in include/pfsolve.h)."""
        _check(load().pf_checkpoint_save(self.handle, os.fsencode(path)))

    def load_checkpoint(self, path: str):
        """Replace the state with a checkpoint of the same nx, ny, nz."""
        _check(load().pf_checkpoint_load(self.handle, os.fsencode(path)))

    def mesh(self, phase: int, iso: float = 0.5):
        """Interface mesh of one phase on the GPU: float32 array [ntri, 3, 3]
        of triangle vertices (cell-index units), in no fixed order.  Counts
        first, then extracts into a device buffer of the exact size."""
        import torch

        lib = load()
        n = C.c_int64()
        empty = A.PfDeviceBuffer(None, 0)
        st = lib.pf_mesh_phase(self.handle, int(phase), float(iso), C.byref(empty), C.byref(n))
        if st not in (A.PF_OK, A.PF_ERR_INVALID_ARG) or (st != A.PF_OK and n.value == 0):
            _check(st)
        buf = torch.empty(max(n.value, 1) * 9, dtype=torch.float32, device="cuda")
        dev = A.PfDeviceBuffer(C.c_void_p(buf.data_ptr()), n.value * 36)
        _check(lib.pf_mesh_phase(self.handle, int(phase), float(iso), C.byref(dev), C.byref(n)))
        return buf[: n.value * 9].cpu().numpy().reshape(-1, 3, 3)

    def diagnostics(self, raise_nonfinite: bool = True) -> dict:
        dg = A.PfDiag()
        st = load().pf_read_fields(self.handle, None, None, C.byref(dg))
        if st != A.PF_OK and (raise_nonfinite or st != A.PF_ERR_NONFINITE):
            _check(st)
        return _diag_dict(dg)


class Pack:
    """Many domains of one precision stepped together by one launch per
    kernel per step, captured in a HIP graph."""

    def __init__(self, prec="fp32", stream=None, max_domains: int = 256):
        h = C.c_void_p()
        _check(load().pf_pack_create(_prec_code(prec), C.c_void_p(_stream_handle(stream)),
                                     int(max_domains), C.byref(h)))
        self._h = h
        self.stream = stream
        self.members: list[Domain] = []

    def add(self, dom: Domain, nsteps: int):
        _check(load().pf_pack_add(self._h, dom.handle, int(nsteps)))
        self.members.append(dom)

    def remove(self, dom: Domain):
        _check(load().pf_pack_remove(self._h, dom.handle))
        self.members.remove(dom)

    def step(self, rounds: int = 1, count_finished: bool = False):
        n = C.c_int32(0)
        _check(load().pf_pack_step(self._h, int(rounds), C.byref(n) if count_finished else None))
        return n.value if count_finished else None

    def remaining(self, dom: Domain) -> int:
        v = C.c_int64()
        _check(load().pf_pack_remaining(self._h, dom.handle, C.byref(v)))
        return v.value

    def sync(self):
        _check(load().pf_pack_sync(self._h))

    def close(self):
        if getattr(self, "_h", None) is not None:
            load().pf_pack_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
