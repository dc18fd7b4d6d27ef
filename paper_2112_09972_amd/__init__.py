"""Python binding of ``libsclbm.so``, the MI355X (gfx950) two-component Shan-Chen
lattice Boltzmann library (arXiv 2112.09972).

Argument marshalling only: every step of the method runs in the HIP kernels of
``csrc/``.  PyTorch provides device memory (the workspace and field tensors) and
the HIP stream.  The module-level ``sclbm_*`` functions mirror the C calls of
``include/sclbm.h`` one to one; :class:`Lattice` bundles a context with its
workspace and stream.  If the library is not built, importing the binding
fails loudly — there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
# SCLBM_LIBRARY selects another build of the library (the debug variant
# libsclbm_debug.so); by default the one next to this file.
LIB_PATH = os.environ.get("SCLBM_LIBRARY") or os.path.join(_PKG, "libsclbm.so")

SCLBM_OK, SCLBM_EINVAL, SCLBM_ESIZE, SCLBM_EHIP, SCLBM_EUNSTABLE, SCLBM_ESTATE = 0, -1, -2, -3, -4, -5
BC = {"periodic": 0, "ghost": 1}
PREC = {"f64": 0, "f32": 1, "f16dev": 2, "bf16dev": 3, "f32d": 4}
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ESIZE", -3: "EHIP", -4: "EUNSTABLE", -5: "ESTATE"}


class SclbmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


class sclbm_config(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("nbox", ctypes.c_int32), ("bc", ctypes.c_int32), ("prec", ctypes.c_int32),
                ("table_len", ctypes.c_int64), ("tau", ctypes.c_double * 2), ("g_ab", ctypes.c_double),
                ("rho_b", ctypes.c_double * 2), ("mach_max", ctypes.c_double)]


class sclbm_droplet_stats(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("volume", ctypes.c_double), ("com", ctypes.c_double * 3),
                ("cov", ctypes.c_double * 6), ("semi_axes", ctypes.c_double * 3),
                ("deformation", ctypes.c_double), ("r_eq", ctypes.c_double)]

    def as_dict(self):
        return dict(step=self.step, volume=self.volume, com=np.array(self.com[:]), cov=np.array(self.cov[:]),
                    semi_axes=np.array(self.semi_axes[:]), deformation=self.deformation, r_eq=self.r_eq)


EXPORTS = [
    "sclbm_workspace_bytes", "sclbm_create", "sclbm_destroy", "sclbm_init_droplet", "sclbm_init_fields",
    "sclbm_set_gradient_table", "sclbm_step", "sclbm_get_step", "sclbm_fields", "sclbm_totals",
    "sclbm_droplet_moments", "sclbm_droplet_from_moments", "sclbm_droplet", "sclbm_velocity_error",
    "sclbm_state_bytes", "sclbm_save", "sclbm_load", "sclbm_set_launch", "sclbm_get_launch", "sclbm_default_launch",
    "sclbm_last_error", "sclbm_step_graph", "sclbm_autotune", "sclbm_droplet_moments_all", "sclbm_mm_integrate",
    "sclbm_droplet_surface_all", "sclbm_deformation_lbm", "sclbm_droplet_mass_all", "sclbm_reinject",
    "sclbm_droplet_moments_all_static", "sclbm_set_gradient", "sclbm_init_uniform", "sclbm_set_health_check",
    "sclbm_mm_semi_axes",
    # droplet-shape surrogate (sclmlp.h)
    "sclmlp_workspace_bytes", "sclmlp_create", "sclmlp_destroy", "sclmlp_set_params", "sclmlp_get_params",
    "sclmlp_get_grads", "sclmlp_set_normalization", "sclmlp_predict", "sclmlp_gradients", "sclmlp_adam",
    "sclmlp_train_step", "sclmlp_get_step", "sclmlp_bad_rows", "sclmlp_last_error",
]


def _load_library():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libsclbm.so is not built (%s); run `python -c \"import __graft_entry__ as g; g.build()\"`"
                          % LIB_PATH)
    # PyTorch brings its own HIP runtime.  Loading it first makes the library bind
    # to that same runtime; loaded the other way round the process holds two HIP
    # and two HSA runtimes, and the library's one finds no device.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    I32, I64, D = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    dp = ctypes.POINTER(ctypes.c_double)
    cfgp = ctypes.POINTER(sclbm_config)
    sig = {
        "sclbm_workspace_bytes": [cfgp, ctypes.POINTER(ctypes.c_size_t)],
        "sclbm_create": [cfgp, P, ctypes.c_size_t, P, ctypes.POINTER(P)],
        "sclbm_destroy": [P],
        "sclbm_init_droplet": [P, I32, dp, D, D, D, D, dp],
        "sclbm_init_fields": [P, I32, P, P, P],
        "sclbm_set_gradient_table": [P, I32, dp, I64, I64],
        "sclbm_set_gradient": [P, I32, dp],
        "sclbm_init_uniform": [P, I32, D, D, dp],
        "sclbm_set_health_check": [P, I64],
        "sclbm_mm_semi_axes": [dp, I64, dp],
        "sclbm_step": [P, I64],
        "sclbm_step_graph": [P, I64],
        "sclbm_autotune": [P, I32, ctypes.POINTER(I32), ctypes.POINTER(I32), ctypes.POINTER(I32),
                           ctypes.POINTER(ctypes.c_float)],
        "sclbm_get_step": [P, ctypes.POINTER(I64)],
        "sclbm_fields": [P, I32, P, P, P],
        "sclbm_totals": [P, I32, dp, dp],
        "sclbm_droplet_moments": [P, I32, P],
        "sclbm_droplet_moments_all": [P, P],
        "sclbm_droplet_moments_all_static": [P, P],
        "sclbm_droplet_surface_all": [P, P],
        "sclbm_deformation_lbm": [D, D, dp],
        "sclbm_droplet_mass_all": [P, P],
        "sclbm_reinject": [P, I32, dp],
        "sclbm_mm_integrate": [P, I64, I64, D, D, I32, I32, P, P, P],
        "sclbm_droplet_from_moments": [dp, dp, I64, ctypes.POINTER(sclbm_droplet_stats)],
        "sclbm_droplet": [P, I32, ctypes.POINTER(sclbm_droplet_stats)],
        "sclbm_velocity_error": [P, I32, dp, dp],
        "sclbm_state_bytes": [P, ctypes.POINTER(ctypes.c_size_t)],
        "sclbm_save": [P, P, ctypes.c_size_t],
        "sclbm_load": [P, P, ctypes.c_size_t],
        "sclbm_set_launch": [P, I32, I32, I32],
        "sclbm_get_launch": [P, ctypes.POINTER(I32), ctypes.POINTER(I32), ctypes.POINTER(I32)],
        "sclbm_default_launch": [cfgp, ctypes.POINTER(I32), ctypes.POINTER(I32), ctypes.POINTER(I32)],
        "sclmlp_workspace_bytes": [I64, ctypes.POINTER(ctypes.c_size_t)],
        "sclmlp_create": [I64, P, ctypes.c_size_t, P, ctypes.POINTER(P)],
        "sclmlp_destroy": [P],
        "sclmlp_set_params": [P, P],
        "sclmlp_get_params": [P, P],
        "sclmlp_get_grads": [P, P],
        "sclmlp_set_normalization": [P, P, P, P, P],
        "sclmlp_predict": [P, P, I64, P],
        "sclmlp_gradients": [P, P, P, P, P, I64, I64, P],
        "sclmlp_adam": [P, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float],
        "sclmlp_train_step": [P, P, P, P, P, I64, I64, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                              P],
        "sclmlp_get_step": [P, ctypes.POINTER(I64)],
        "sclmlp_bad_rows": [P, ctypes.POINTER(I64)],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    for name in ("sclbm_last_error", "sclmlp_last_error"):
        getattr(lib, name).argtypes = []
        getattr(lib, name).restype = ctypes.c_char_p
    return lib


class _LazyLib:
    """Loads libsclbm.so on first use (so that the build step can import this
    package before the library exists); raises ImportError if it is missing."""
    _handle = None

    def __getattr__(self, name):
        if _LazyLib._handle is None:
            _LazyLib._handle = _load_library()
        return getattr(_LazyLib._handle, name)


_lib = _LazyLib()


def load():
    """Load the library now (ImportError if it is not built); returns the ctypes handle."""
    _lib.sclbm_last_error
    return _LazyLib._handle


def _check(status: int):
    if status != SCLBM_OK:
        raise SclbmError(status, _lib.sclbm_last_error().decode())


def _dvec(values, n):
    arr = (ctypes.c_double * n)(*[float(v) for v in np.asarray(values, dtype=np.float64).reshape(n)])
    return arr


# ---- one-to-one wrappers of the C calls -------------------------------------------------------

def sclbm_workspace_bytes(cfg: sclbm_config) -> int:
    b = ctypes.c_size_t()
    _check(_lib.sclbm_workspace_bytes(ctypes.byref(cfg), ctypes.byref(b)))
    return b.value


def sclbm_create(cfg: sclbm_config, dev_workspace: int, nbytes: int, stream: int):
    h = ctypes.c_void_p()
    _check(_lib.sclbm_create(ctypes.byref(cfg), ctypes.c_void_p(dev_workspace), nbytes, ctypes.c_void_p(stream),
                             ctypes.byref(h)))
    return h


def sclbm_destroy(ctx):
    _check(_lib.sclbm_destroy(ctx))


def sclbm_init_droplet(ctx, box, center, radius, width, rho_in, rho_out, A0=None):
    a = _dvec(A0, 9) if A0 is not None else None
    _check(_lib.sclbm_init_droplet(ctx, box, _dvec(center, 3), radius, width, rho_in, rho_out, a))


def sclbm_init_fields(ctx, box, rho_a_ptr, rho_b_ptr, u_ptr=None):
    _check(_lib.sclbm_init_fields(ctx, box, ctypes.c_void_p(rho_a_ptr), ctypes.c_void_p(rho_b_ptr),
                                  ctypes.c_void_p(u_ptr) if u_ptr else None))


def sclbm_set_gradient_table(ctx, box, A_rows: np.ndarray, first_step: int):
    a = np.ascontiguousarray(np.asarray(A_rows, dtype=np.float64).reshape(-1, 9))
    _check(_lib.sclbm_set_gradient_table(ctx, box, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                         int(first_step), a.shape[0]))


def sclbm_set_gradient(ctx, box, A):
    _check(_lib.sclbm_set_gradient(ctx, box, _dvec(A, 9)))


def sclbm_init_uniform(ctx, box, rho_a, rho_b, u0=None):
    _check(_lib.sclbm_init_uniform(ctx, box, float(rho_a), float(rho_b), _dvec(u0, 3) if u0 is not None else None))


def sclbm_set_health_check(ctx, every: int):
    _check(_lib.sclbm_set_health_check(ctx, int(every)))


def sclbm_mm_semi_axes(M) -> np.ndarray:
    """Semi-axes over R of Maffettone-Minale tensors M[..., 3, 3], descending: shape [..., 3]."""
    M = np.asarray(M, dtype=np.float64)
    assert M.shape[-2:] == (3, 3)
    m = np.ascontiguousarray(M.reshape(-1, 9))
    out = np.zeros((m.shape[0], 3))
    _check(_lib.sclbm_mm_semi_axes(m.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), m.shape[0],
                                   out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out.reshape(M.shape[:-2] + (3,))


def sclbm_step(ctx, nsteps: int):
    _check(_lib.sclbm_step(ctx, int(nsteps)))


def sclbm_step_graph(ctx, nsteps: int):
    _check(_lib.sclbm_step_graph(ctx, int(nsteps)))


def sclbm_autotune(ctx, trial_steps: int):
    """Returns (tile_rows, zchunk, tile_waves, best_ms)."""
    t = ctypes.c_int32()
    z = ctypes.c_int32()
    w = ctypes.c_int32()
    ms = ctypes.c_float()
    _check(_lib.sclbm_autotune(ctx, int(trial_steps), ctypes.byref(t), ctypes.byref(z), ctypes.byref(w),
                               ctypes.byref(ms)))
    return t.value, z.value, w.value, ms.value


def sclbm_get_step(ctx) -> int:
    s = ctypes.c_int64()
    _check(_lib.sclbm_get_step(ctx, ctypes.byref(s)))
    return s.value


def sclbm_fields(ctx, box, rho_a_ptr, rho_b_ptr, u_ptr=None):
    _check(_lib.sclbm_fields(ctx, box, ctypes.c_void_p(rho_a_ptr), ctypes.c_void_p(rho_b_ptr),
                             ctypes.c_void_p(u_ptr) if u_ptr else None))


def sclbm_totals(ctx, box):
    m = (ctypes.c_double * 2)()
    p = (ctypes.c_double * 3)()
    st = _lib.sclbm_totals(ctx, box, m, p)
    if st not in (SCLBM_OK, SCLBM_EUNSTABLE):
        _check(st)
    return np.array(m[:]), np.array(p[:]), st


def sclbm_droplet_moments(ctx, box, dev_out_ptr):
    _check(_lib.sclbm_droplet_moments(ctx, box, ctypes.c_void_p(dev_out_ptr)))


def sclbm_droplet_moments_all(ctx, dev_out_ptr):
    _check(_lib.sclbm_droplet_moments_all(ctx, ctypes.c_void_p(dev_out_ptr)))


def sclbm_droplet_moments_all_static(ctx, dev_out_ptr):
    _check(_lib.sclbm_droplet_moments_all_static(ctx, ctypes.c_void_p(dev_out_ptr)))


def sclbm_droplet_surface_all(ctx, dev_out_ptr):
    _check(_lib.sclbm_droplet_surface_all(ctx, ctypes.c_void_p(dev_out_ptr)))


def sclbm_deformation_lbm(area, volume) -> float:
    d = ctypes.c_double()
    _check(_lib.sclbm_deformation_lbm(float(area), float(volume), ctypes.byref(d)))
    return d.value


def sclbm_droplet_mass_all(ctx, dev_out_ptr):
    _check(_lib.sclbm_droplet_mass_all(ctx, ctypes.c_void_p(dev_out_ptr)))


def sclbm_reinject(ctx, box, target_mass):
    t = np.ascontiguousarray(np.atleast_1d(np.asarray(target_mass, dtype=np.float64)))
    _check(_lib.sclbm_reinject(ctx, int(box), t.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))


def sclbm_droplet_from_moments(moments, center, step=0) -> dict:
    out = sclbm_droplet_stats()
    _check(_lib.sclbm_droplet_from_moments(_dvec(moments, 10), _dvec(center, 3), int(step), ctypes.byref(out)))
    return out.as_dict()


def sclbm_droplet(ctx, box) -> dict:
    out = sclbm_droplet_stats()
    _check(_lib.sclbm_droplet(ctx, box, ctypes.byref(out)))
    return out.as_dict()


def sclbm_velocity_error(ctx, box, A) -> float:
    e = ctypes.c_double()
    _check(_lib.sclbm_velocity_error(ctx, box, _dvec(A, 9), ctypes.byref(e)))
    return e.value


def sclbm_state_bytes(ctx) -> int:
    b = ctypes.c_size_t()
    _check(_lib.sclbm_state_bytes(ctx, ctypes.byref(b)))
    return b.value


def sclbm_save(ctx, buf: np.ndarray):
    _check(_lib.sclbm_save(ctx, buf.ctypes.data_as(ctypes.c_void_p), buf.nbytes))


def sclbm_load(ctx, buf: np.ndarray):
    _check(_lib.sclbm_load(ctx, buf.ctypes.data_as(ctypes.c_void_p), buf.nbytes))


def sclbm_set_launch(ctx, tile_rows: int, zchunk: int, tile_waves: int = 1):
    _check(_lib.sclbm_set_launch(ctx, int(tile_rows), int(zchunk), int(tile_waves)))


def sclbm_get_launch(ctx):
    """Returns (tile_rows, zchunk, tile_waves)."""
    t = ctypes.c_int32()
    z = ctypes.c_int32()
    w = ctypes.c_int32()
    _check(_lib.sclbm_get_launch(ctx, ctypes.byref(t), ctypes.byref(z), ctypes.byref(w)))
    return t.value, z.value, w.value


def sclbm_default_launch(cfg: sclbm_config):
    """The launch shape a context with this configuration starts with,
    computed on the host: (tile_rows, zchunk, tile_waves)."""
    t = ctypes.c_int32()
    z = ctypes.c_int32()
    w = ctypes.c_int32()
    _check(_lib.sclbm_default_launch(ctypes.byref(cfg), ctypes.byref(t), ctypes.byref(z), ctypes.byref(w)))
    return t.value, z.value, w.value


def sclbm_mm_integrate(dev_A_ptr, ntraj, nrows, tau_d, chi, substeps, record_every, dev_M0_ptr, dev_M_ptr, stream):
    _check(_lib.sclbm_mm_integrate(ctypes.c_void_p(dev_A_ptr), int(ntraj), int(nrows), float(tau_d), float(chi),
                                   int(substeps), int(record_every), ctypes.c_void_p(dev_M0_ptr) if dev_M0_ptr else None,
                                   ctypes.c_void_p(dev_M_ptr), ctypes.c_void_p(stream)))


def mm_integrate(A_rows, tau_d, chi=1.0, substeps=1, record_every=1, M0=None, device="cuda:0"):
    """Torch convenience wrapper: A_rows (ntraj, nrows, 9) -> M (ntraj, nrec, 3, 3), on the GPU."""
    import torch
    A = torch.as_tensor(np.ascontiguousarray(A_rows, dtype=np.float64)).to(device)
    ntraj, nrows = A.shape[0], A.shape[1]
    nrec = 1 + (nrows - 1) // record_every
    out = torch.empty((ntraj, nrec, 9), dtype=torch.float64, device=device)
    m0 = None if M0 is None else torch.as_tensor(np.ascontiguousarray(M0, dtype=np.float64)).to(device)
    stream = torch.cuda.current_stream(device)
    sclbm_mm_integrate(A.data_ptr(), ntraj, nrows, tau_d, chi, substeps, record_every,
                       m0.data_ptr() if m0 is not None else None, out.data_ptr(), stream.cuda_stream)
    stream.synchronize()
    return out.reshape(ntraj, nrec, 3, 3)


def sclbm_last_error() -> str:
    return _lib.sclbm_last_error().decode()


# ---- convenience object ------------------------------------------------------------------------

class Lattice:
    """A context plus its torch-owned workspace and stream.

    Boxes are (nz, ny, nx) arrays of nodes; fields come back as torch FP64
    tensors on the device.  ``bc`` is "ghost" or "periodic"; ``prec`` one of
    "f64", "f32", "f16dev", "bf16dev".
    """

    def __init__(self, nx, ny, nz, *, nbox=1, bc="ghost", prec="f64", table_len=1, tau=(1.0, 1.0), g_ab=0.0,
                 rho_b=(0.04, 1.0), mach_max=0.0, device="cuda:0", stream=None):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.shape = (nz, ny, nx)
        self.nx, self.ny, self.nz, self.nbox = nx, ny, nz, nbox
        self.N = nx * ny * nz
        self.xc = np.array([(nx - 1) / 2.0, (ny - 1) / 2.0, (nz - 1) / 2.0])
        self.cfg = sclbm_config(nx=nx, ny=ny, nz=nz, nbox=nbox, bc=BC[bc], prec=PREC[prec],
                                table_len=int(table_len), tau=(ctypes.c_double * 2)(*tau), g_ab=float(g_ab),
                                rho_b=(ctypes.c_double * 2)(*rho_b), mach_max=float(mach_max))
        nbytes = sclbm_workspace_bytes(self.cfg)
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.ctx = sclbm_create(self.cfg, self.workspace.data_ptr(), nbytes, self.stream.cuda_stream)
        self._mom = torch.empty(10, dtype=torch.float64, device=self.device)

    def close(self):
        if getattr(self, "ctx", None):
            self.stream.synchronize()
            sclbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _sync_torch(self):
        # torch-allocated inputs are produced on torch's current stream
        self.stream.wait_stream(self.torch.cuda.current_stream(self.device))

    @property
    def step_count(self) -> int:
        return sclbm_get_step(self.ctx)

    def init_droplet(self, center, radius, width, rho_in, rho_out, A0=None, box=-1):
        sclbm_init_droplet(self.ctx, box, center, radius, width, rho_in, rho_out, A0)

    def init_fields(self, rho_a, rho_b, u=None, box=0):
        t = self.torch
        ra = t.as_tensor(np.array(np.broadcast_to(rho_a, self.shape), dtype=np.float64)).to(self.device)
        rb = t.as_tensor(np.array(np.broadcast_to(rho_b, self.shape), dtype=np.float64)).to(self.device)
        uu = None
        if u is not None:
            u = np.asarray(u, dtype=np.float64)
            if u.shape == (3,):
                u = u.reshape(3, 1, 1, 1)
            uu = t.as_tensor(np.array(np.broadcast_to(u, (3,) + self.shape), dtype=np.float64)).to(self.device)
        self._sync_torch()
        sclbm_init_fields(self.ctx, box, ra.data_ptr(), rb.data_ptr(), uu.data_ptr() if uu is not None else None)
        self.stream.synchronize()

    def init_uniform(self, rho_a, rho_b, u0=None, box=-1):
        sclbm_init_uniform(self.ctx, box, rho_a, rho_b, u0)

    def set_gradient(self, A, box=-1):
        sclbm_set_gradient(self.ctx, box, A)

    def set_health_check(self, every):
        sclbm_set_health_check(self.ctx, every)

    def set_gradient_table(self, A_rows, first_step=0, box=0):
        sclbm_set_gradient_table(self.ctx, box, A_rows, first_step)

    def step(self, nsteps):
        sclbm_step(self.ctx, nsteps)

    def step_graph(self, nsteps):
        """nsteps (even) fused launches replayed from a captured hipGraph."""
        sclbm_step_graph(self.ctx, nsteps)

    def autotune(self, trial_steps=20, cache=True):
        """Pick the fastest launch shape (clobbers the populations: call before
        an init).  Results are cached in $XDG_CACHE_HOME/sclbm/tuning.json keyed
        by device, box shape, boxes, precision and boundary mode."""
        import json
        key = "%s|%dx%dx%d|%d|%d|%d|rowtiles5" % (self.torch.cuda.get_device_properties(self.device).name, self.nx,
                                                 self.ny, self.nz, self.nbox, self.cfg.prec, self.cfg.bc)
        path = os.path.join(os.environ.get("XDG_CACHE_HOME", os.path.expanduser("~/.cache")), "sclbm", "tuning.json")
        table = {}
        if cache and os.path.exists(path):
            try:
                with open(path) as fh:
                    table = json.load(fh)
            except (OSError, ValueError):
                table = {}
        if key in table:
            ty, zc, wx = table[key]["tile_rows"], table[key]["zchunk"], table[key]["tile_waves"]
            self.set_launch(ty, zc, wx)
            return ty, zc, wx, table[key]["ms"]
        ty, zc, wx, ms = sclbm_autotune(self.ctx, trial_steps)
        if cache:
            table[key] = {"tile_rows": ty, "zchunk": zc, "tile_waves": wx, "ms": ms}
            try:
                os.makedirs(os.path.dirname(path), exist_ok=True)
                with open(path, "w") as fh:
                    json.dump(table, fh, indent=1)
            except OSError:
                pass
        return ty, zc, wx, ms

    def synchronize(self):
        self.stream.synchronize()

    def fields(self, box=0, velocity=True):
        t = self.torch
        ra = t.empty(self.shape, dtype=t.float64, device=self.device)
        rb = t.empty(self.shape, dtype=t.float64, device=self.device)
        u = t.empty((3,) + self.shape, dtype=t.float64, device=self.device) if velocity else None
        self._sync_torch()
        sclbm_fields(self.ctx, box, ra.data_ptr(), rb.data_ptr(), u.data_ptr() if velocity else None)
        self.stream.synchronize()
        return (ra, rb, u) if velocity else (ra, rb)

    def totals(self, box=0, check=True):
        m, p, st = sclbm_totals(self.ctx, box)
        if check and st != SCLBM_OK:
            _check(st)
        return m, p

    def droplet(self, box=0) -> dict:
        return sclbm_droplet(self.ctx, box)

    def droplet_moments(self, out, box=0):
        """Enqueue the 10 indicator moments of ``box`` into the device tensor ``out``."""
        sclbm_droplet_moments(self.ctx, box, out.data_ptr())

    def droplet_moments_all(self, out):
        """Enqueue the 10 indicator moments of every box into the device tensor out[nbox][10]."""
        assert out.shape == (self.nbox, 10) and out.is_contiguous()
        sclbm_droplet_moments_all(self.ctx, out.data_ptr())

    def droplet_surface_all(self, out):
        """Enqueue {area, volume} of every box's droplet into the device tensor out[nbox][2]."""
        assert out.shape == (self.nbox, 2) and out.is_contiguous()
        sclbm_droplet_surface_all(self.ctx, out.data_ptr())

    def droplet_surface(self, box=0):
        """(area, volume, D_LBM) of one box's droplet (synchronises)."""
        out = self.torch.empty((self.nbox, 2), dtype=self.torch.float64, device=self.device)
        self._sync_torch()
        self.droplet_surface_all(out)
        self.stream.synchronize()
        area, vol = (float(v) for v in out[box].cpu())
        return area, vol, sclbm_deformation_lbm(area, vol)

    def droplet_mass(self):
        """Droplet mass of every box (numpy, synchronises)."""
        out = self.torch.empty(self.nbox, dtype=self.torch.float64, device=self.device)
        self._sync_torch()
        sclbm_droplet_mass_all(self.ctx, out.data_ptr())
        self.stream.synchronize()
        return out.cpu().numpy()

    def reinject(self, target_mass, box=-1):
        """Scale component A in the droplet(s) so that the droplet mass becomes the target."""
        sclbm_reinject(self.ctx, box, target_mass)

    def velocity_error(self, A, box=0) -> float:
        return sclbm_velocity_error(self.ctx, box, A)

    def save(self) -> np.ndarray:
        buf = np.empty(sclbm_state_bytes(self.ctx), dtype=np.uint8)
        sclbm_save(self.ctx, buf)
        return buf

    def load(self, buf: np.ndarray):
        sclbm_load(self.ctx, np.ascontiguousarray(buf))

    def set_launch(self, tile_rows, zchunk, tile_waves=1):
        """Step-kernel tile of tile_rows rows x tile_waves 64-node columns and
        z-chunk of zchunk planes; (tile_rows, tile_waves) in (4, 1), (8, 1), (4, 2).
        Speed only: results are bitwise the same for every shape."""
        sclbm_set_launch(self.ctx, tile_rows, zchunk, tile_waves)

    def get_launch(self):
        return sclbm_get_launch(self.ctx)
