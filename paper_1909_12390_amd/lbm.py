"""ctypes binding of include/lbm.h (argument marshalling only).

Every step of the model runs in the HIP library libpaper_lbm.so; this module only
converts Python/NumPy/torch arguments into the C structures and device pointers
the ABI takes.  If the library is not built, every call raises: there is no
fallback implementation.

torch is used for device memory (the caller-owned workspace and field tensors)
and for the current HIP stream.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_int, c_size_t, c_void_p

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpaper_lbm.so")

# enum values of include/lbm.h
LBM_OK, LBM_ERR_ARG, LBM_ERR_DOMAIN, LBM_ERR_HIP, LBM_ERR_NOCONVERGE, LBM_ERR_SINGLEPHASE, LBM_ERR_UNSUPPORTED = \
    0, -1, -2, -3, -4, -5, -6
LATTICES = {"D2Q9": 0, "D3Q19": 1}
COLLISIONS = {"bgk": 0, "mrt": 1}
FORCINGS = {"guo": 0, "edm": 1}
STORAGES = {"f64": 0, "f32": 1, "f16": 2}
SCHEDULES = {"two_pass": 0, "blocked": 1, "overlap": 2}
MAX_NC = 4
MAX_Q = 19
Q_OF = {"D2Q9": 9, "D3Q19": 19}
D_OF = {"D2Q9": 2, "D3Q19": 3}

# every function declared in include/lbm.h
EXPORTED = ["lbm_workspace_bytes", "lbm_init", "lbm_step", "lbm_step_timed", "lbm_moments", "lbm_moments_noalloc",
            "lbm_get_populations", "lbm_stream_copy",
            "lbm_set_populations", "lbm_check", "lbm_clear_error", "lbm_destroy", "lbm_last_error",
            "lbm_critical", "lbm_fugacity", "lbm_flash", "lbm_bubble_pressure", "lbm_dew_pressure",
            "lbm_batch_layout", "lbm_batch_init", "lbm_batch_step", "lbm_batch_fields", "lbm_batch_check",
            "lbm_batch_box_errors", "lbm_batch_destroy", "lbm_adjoint_workspace", "lbm_step_adjoint",
            "lbm_adjoint", "lbm_eos_param_grad", "lbm_set_gamma", "lbm_batch_set_gamma", "lbm_set_solid",
            "lbm_set_graph_steps"]


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"lbm status {code}: {msg}")
        self.code = code


class LbmMixture(ctypes.Structure):
    _fields_ = [("nc", c_int), ("R", c_double), ("a", c_double * MAX_NC), ("b", c_double * MAX_NC),
                ("omega", c_double * MAX_NC), ("M", c_double * MAX_NC), ("k", (c_double * MAX_NC) * MAX_NC)]


class LbmParams(ctypes.Structure):
    _fields_ = [("lattice", c_int), ("nx", c_int), ("ny", c_int), ("nz", c_int), ("collision", c_int),
                ("forcing", c_int), ("storage", c_int), ("schedule", c_int), ("slab_planes", c_int), ("T", c_double),
                ("tau", c_double), ("G", c_double), ("beta", c_double), ("gamma", c_double * MAX_NC),
                ("mrt_s", c_double * MAX_Q), ("accel", c_double * 3), ("p_flash", c_double),
                ("z_flash", c_double * MAX_NC)]


class LbmFlashResult(ctypes.Structure):
    _fields_ = [("V", c_double), ("x", c_double * MAX_NC), ("y", c_double * MAX_NC), ("K", c_double * MAX_NC),
                ("Zl", c_double), ("Zv", c_double), ("rho_l", c_double), ("rho_v", c_double),
                ("rbar_l", c_double * MAX_NC), ("rbar_v", c_double * MAX_NC), ("gamma", c_double * MAX_NC),
                ("fug_l", c_double * MAX_NC), ("fug_v", c_double * MAX_NC), ("residual", c_double),
                ("iterations", c_int)]


class LbmBox(ctypes.Structure):
    _fields_ = [("mix", LbmMixture), ("nx", c_int), ("ny", c_int), ("nz", c_int), ("T", c_double),
                ("tau", c_double), ("G", c_double), ("beta", c_double), ("gamma", c_double * MAX_NC),
                ("solid", c_void_p), ("psi_wall", c_double)]


class LbmBatchParams(ctypes.Structure):
    _fields_ = [("lattice", c_int), ("collision", c_int), ("forcing", c_int), ("storage", c_int),
                ("tile", c_int), ("graph_steps", c_int), ("grid", c_int), ("mrt_s", c_double * MAX_Q),
                ("accel", c_double * 3), ("fused", c_int)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libpaper_lbm.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is None:
        # torch first: the library and torch must share one HIP runtime in the
        # process, and the first one loaded is the one both use
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise LbmError(LBM_ERR_UNSUPPORTED,
                           f"{LIB_PATH} is not built (python -m paper_1909_12390_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        dp = POINTER(c_double)
        L.lbm_workspace_bytes.argtypes = [POINTER(LbmMixture), POINTER(LbmParams), POINTER(c_size_t)]
        L.lbm_init.argtypes = [POINTER(LbmMixture), POINTER(LbmParams), c_void_p, c_size_t, c_void_p, c_void_p,
                               c_void_p, POINTER(c_void_p)]
        L.lbm_step.argtypes = [c_void_p, c_int]
        L.lbm_step_timed.argtypes = [c_void_p, c_int, dp]
        L.lbm_moments.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, dp]
        L.lbm_moments_noalloc.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, dp]
        L.lbm_stream_copy.argtypes = [c_void_p, c_void_p, c_size_t, c_int, c_void_p]
        L.lbm_get_populations.argtypes = [c_void_p, c_void_p]
        L.lbm_set_populations.argtypes = [c_void_p, c_void_p]
        L.lbm_check.argtypes = [c_void_p]
        L.lbm_clear_error.argtypes = [c_void_p]
        L.lbm_destroy.argtypes = [c_void_p]
        L.lbm_destroy.restype = None
        L.lbm_last_error.restype = ctypes.c_char_p
        L.lbm_critical.argtypes = [POINTER(LbmMixture), dp, dp]
        L.lbm_fugacity.argtypes = [POINTER(LbmMixture), c_double, c_int, dp, dp, dp, dp, dp]
        L.lbm_flash.argtypes = [POINTER(LbmMixture), c_double, c_double, dp, POINTER(LbmFlashResult)]
        L.lbm_bubble_pressure.argtypes = [POINTER(LbmMixture), c_double, dp, dp]
        L.lbm_dew_pressure.argtypes = [POINTER(LbmMixture), c_double, dp, dp]
        L.lbm_batch_layout.argtypes = [POINTER(LbmBox), c_int, POINTER(LbmBatchParams), POINTER(c_size_t),
                                       POINTER(c_size_t), POINTER(c_size_t)]
        L.lbm_batch_init.argtypes = [POINTER(LbmBox), c_int, POINTER(LbmBatchParams), c_void_p, c_size_t, c_void_p,
                                     c_void_p, POINTER(c_void_p)]
        L.lbm_batch_step.argtypes = [c_void_p, c_int]
        L.lbm_batch_fields.argtypes = [c_void_p, c_void_p, c_void_p]
        L.lbm_batch_check.argtypes = [c_void_p]
        L.lbm_batch_box_errors.argtypes = [c_void_p, POINTER(c_int)]
        L.lbm_batch_destroy.argtypes = [c_void_p]
        L.lbm_batch_destroy.restype = None
        L.lbm_adjoint_workspace.argtypes = [c_void_p, c_int, c_int, POINTER(c_size_t)]
        L.lbm_step_adjoint.argtypes = [c_void_p, c_void_p, c_void_p, dp, dp, c_void_p, c_size_t]
        L.lbm_adjoint.argtypes = [c_void_p, c_int, c_int, c_void_p, dp, c_void_p, c_size_t, dp, dp, dp, dp, dp]
        L.lbm_eos_param_grad.argtypes = [POINTER(LbmMixture), c_double, dp, dp, dp, dp, dp]
        L.lbm_set_gamma.argtypes = [c_void_p, dp]
        L.lbm_batch_set_gamma.argtypes = [c_void_p, c_int, dp]
        L.lbm_set_solid.argtypes = [c_void_p, c_void_p, c_double]
        L.lbm_set_graph_steps.argtypes = [c_void_p, c_int]
        for name in EXPORTED:
            f = getattr(L, name)
            if name not in ("lbm_destroy", "lbm_last_error", "lbm_batch_destroy"):
                f.restype = c_int
        _lib = L
    return _lib


def _check(code: int):
    if code != LBM_OK:
        raise LbmError(code, lib().lbm_last_error().decode())


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(POINTER(c_double))


def mixture_struct(mix: dict) -> LbmMixture:
    m = LbmMixture()
    nc = len(mix["a"])
    m.nc = nc
    m.R = float(mix.get("R", 1.0))
    for i in range(nc):
        m.a[i] = float(mix["a"][i])
        m.b[i] = float(mix["b"][i])
        m.omega[i] = float(mix["omega"][i])
        m.M[i] = float(mix["M"][i])
        for j in range(nc):
            m.k[i][j] = float(np.asarray(mix["k"])[i, j])
    return m


# ---------------------------------------------------------------------------
# thermodynamics (host float64 in the library)
# ---------------------------------------------------------------------------

def lbm_critical(mix: dict):
    m = mixture_struct(mix)
    Tc = np.zeros(m.nc)
    pc = np.zeros(m.nc)
    _check(lib().lbm_critical(ctypes.byref(m), _dptr(Tc), _dptr(pc)))
    return Tc, pc


def lbm_fugacity(mix: dict, T: float, n: np.ndarray):
    """n: molar densities [nstates, nc].  Returns dict p, Z, lnphi, fug."""
    m = mixture_struct(mix)
    n = np.ascontiguousarray(np.atleast_2d(n), dtype=np.float64)
    ns = n.shape[0]
    p = np.zeros(ns)
    Z = np.zeros(ns)
    lp = np.zeros((ns, m.nc))
    fug = np.zeros((ns, m.nc))
    _check(lib().lbm_fugacity(ctypes.byref(m), float(T), ns, _dptr(n), _dptr(p), _dptr(Z), _dptr(lp), _dptr(fug)))
    return {"p": p, "Z": Z, "lnphi": lp, "fug": fug}


def lbm_pressure(mix: dict, T: float, n: np.ndarray) -> np.ndarray:
    """p_EOS of molar-density states n[nstates, nc]; nan where b_m rho~ >= 1."""
    m = mixture_struct(mix)
    n = np.ascontiguousarray(np.atleast_2d(n), dtype=np.float64)
    out = np.full(n.shape[0], np.nan)
    p = np.zeros(1)
    for i in range(n.shape[0]):
        code = lib().lbm_fugacity(ctypes.byref(m), float(T), 1, _dptr(np.ascontiguousarray(n[i:i + 1])),
                                  _dptr(p), None, None, None)
        if code == LBM_OK:
            out[i] = p[0]
        elif code != LBM_ERR_DOMAIN:
            _check(code)
    return out


class FlashResult:
    def __init__(self, r: LbmFlashResult, nc: int):
        for name in ("V", "Zl", "Zv", "rho_l", "rho_v", "residual", "iterations"):
            setattr(self, name, getattr(r, name))
        for name in ("x", "y", "K", "rbar_l", "rbar_v", "gamma", "fug_l", "fug_v"):
            setattr(self, name, np.array(getattr(r, name)[:nc]))


def lbm_flash(mix: dict, T: float, p: float, z) -> FlashResult:
    m = mixture_struct(mix)
    zz = np.ascontiguousarray(z, dtype=np.float64)
    r = LbmFlashResult()
    _check(lib().lbm_flash(ctypes.byref(m), float(T), float(p), _dptr(zz), ctypes.byref(r)))
    return FlashResult(r, m.nc)


def lbm_bubble_pressure(mix: dict, T: float, z) -> float:
    m = mixture_struct(mix)
    zz = np.ascontiguousarray(z, dtype=np.float64)
    out = np.zeros(1)
    _check(lib().lbm_bubble_pressure(ctypes.byref(m), float(T), _dptr(zz), _dptr(out)))
    return float(out[0])


def lbm_dew_pressure(mix: dict, T: float, z) -> float:
    m = mixture_struct(mix)
    zz = np.ascontiguousarray(z, dtype=np.float64)
    out = np.zeros(1)
    _check(lib().lbm_dew_pressure(ctypes.byref(m), float(T), _dptr(zz), _dptr(out)))
    return float(out[0])


def stream_copy(dst, src, nbytes: int, grid: int = 0, stream=None):
    """lbm_stream_copy between two device tensors (the measured bandwidth ceiling);
    enqueued on `stream` (a torch stream; None = the current one)."""
    import torch
    for name, t in (("dst", dst), ("src", src)):
        if not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"stream_copy: {name} must be a contiguous device tensor")
        if int(nbytes) > t.numel() * t.element_size():
            raise ValueError(f"stream_copy: {nbytes} bytes exceed {name} ({t.numel() * t.element_size()} bytes)")
    st = torch.cuda.current_stream() if stream is None else stream
    _check(lib().lbm_stream_copy(c_void_p(dst.data_ptr()), c_void_p(src.data_ptr()), int(nbytes), int(grid),
                                 c_void_p(st.cuda_stream)))


class LibThermo:
    """The library's thermodynamics through the backend interface of inputs.py."""

    def critical_temperature(self, mix):
        return lbm_critical(mix)[0]

    def bubble_pressure(self, mix, T, z):
        return lbm_bubble_pressure(mix, T, z)

    def dew_pressure(self, mix, T, z):
        return lbm_dew_pressure(mix, T, z)

    def flash(self, mix, T, p, z):
        return lbm_flash(mix, T, p, z)

    def pressure(self, mix, T, n):
        return lbm_pressure(mix, T, n)


# ---------------------------------------------------------------------------
# time stepping on the device
# ---------------------------------------------------------------------------

def params_struct(lattice, shape, T, tau, beta, gamma, collision="bgk", forcing="guo", storage="f64",
                  schedule="two_pass", mrt_s=None, accel=None, G=-1.0, slab_planes=0, p_flash=None,
                  z_flash=None) -> LbmParams:
    """gamma None: left zero, so that lbm_init takes it from the flash at (T, p_flash, z_flash)."""
    p = LbmParams()
    p.lattice = LATTICES[lattice]
    if lattice == "D2Q9":
        ny, nx = shape
        nz = 1
    else:
        nz, ny, nx = shape
    p.nx, p.ny, p.nz = int(nx), int(ny), int(nz)
    p.collision = COLLISIONS[collision]
    p.forcing = FORCINGS[forcing]
    p.storage = STORAGES[storage]
    p.schedule = SCHEDULES[schedule]
    p.slab_planes = int(slab_planes)
    p.T = float(T)
    p.tau = float(tau)
    p.G = float(G)
    p.beta = float(beta)
    if gamma is None:
        if p_flash is None or z_flash is None:
            raise ValueError("gamma=None needs p_flash and z_flash (the flash that supplies gamma)")
        p.p_flash = float(p_flash)
        for i, z in enumerate(z_flash):
            p.z_flash[i] = float(z)
    else:
        for i, g in enumerate(gamma):
            p.gamma[i] = float(g)
    if mrt_s is not None:
        for k, s in enumerate(mrt_s):
            p.mrt_s[k] = float(s)
    if accel is not None:
        for d, g in enumerate(accel):
            p.accel[d] = float(g)
    return p


class LbmContext:
    """One simulation box on the current HIP device (one lbm_ctx).

    rho0: initial cell-volume densities (nc, *shape), float64 (NumPy or torch).
    u0  : optional initial velocity (D, *shape).
    gamma: volatility coefficients, or None to have lbm_init take them from the
    two-phase flash at (T, p_flash, z_flash) (Eq. gamma).
    solid, psi_wall: optional solid-cell mask (*shape, bool) and the wetting psi of
    the walls (lbm_set_solid), applied right after the initial state.
    graph_steps > 0: step() replays HIP graphs of that many steps (lbm_set_graph_steps);
    the context then runs on its own (default-priority) stream, and every call that
    hands tensors to or from torch orders that stream against torch's current one.
    """

    def __init__(self, mix: dict, lattice: str, shape, T, tau, beta, gamma, rho0, u0=None,
                 collision="bgk", forcing="guo", storage="f64", schedule="two_pass", mrt_s=None,
                 accel=None, G=-1.0, slab_planes=0, device="cuda", solid=None, psi_wall=0.0, graph_steps=0,
                 p_flash=None, z_flash=None):
        import torch
        self.torch = torch
        self.lattice = lattice
        self.shape = tuple(int(s) for s in shape)
        self.nc = len(mix["a"])
        self.Q = Q_OF[lattice]
        self.D = D_OF[lattice]
        self.cells = int(np.prod(self.shape))
        self._mix = mixture_struct(mix)
        self._prm = params_struct(lattice, self.shape, T, tau, beta, gamma, collision, forcing, storage,
                                  schedule, mrt_s, accel, G, slab_planes, p_flash, z_flash)
        nbytes = c_size_t(0)
        _check(lib().lbm_workspace_bytes(ctypes.byref(self._mix), ctypes.byref(self._prm), ctypes.byref(nbytes)))
        self.workspace = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=device)
        base = self.workspace.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        rho0_t = self._to_device(rho0, (self.nc,) + self.shape)
        u0_t = None if u0 is None else self._to_device(u0, (self.D,) + self.shape)
        self._own_stream = graph_steps > 0
        if self._own_stream:
            self.stream = torch.cuda.Stream(device=self.workspace.device)
            self.stream.wait_stream(torch.cuda.current_stream(self.workspace.device))
        else:
            self.stream = torch.cuda.current_stream(self.workspace.device)
        ctx = c_void_p()
        _check(lib().lbm_init(ctypes.byref(self._mix), ctypes.byref(self._prm), c_void_p(self._ws_ptr),
                              c_size_t(int(nbytes.value)), c_void_p(rho0_t.data_ptr()),
                              None if u0_t is None else c_void_p(u0_t.data_ptr()),
                              c_void_p(self.stream.cuda_stream), ctypes.byref(ctx)))
        self._ctx = ctx
        self.stream.synchronize()     # the init kernel has read rho0_t / u0_t
        self._keep = None
        if solid is not None:
            self.set_solid(solid, psi_wall)
        if graph_steps > 0:
            _check(lib().lbm_set_graph_steps(self._ctx, int(graph_steps)))

    def _inputs_ready(self):
        """Own stream: wait for torch's current stream (tensors it just wrote)."""
        if self._own_stream:
            self.stream.wait_stream(self.torch.cuda.current_stream(self.workspace.device))

    def _outputs_ready(self):
        """Own stream: torch's current stream waits for the library's writes."""
        if self._own_stream:
            self.torch.cuda.current_stream(self.workspace.device).wait_stream(self.stream)

    def set_solid(self, solid, psi_wall=0.0):
        """Solid walls (halfway bounce-back, psi = psi_wall on solid cells); None
        removes them.  Cells that stay fluid keep their populations."""
        if solid is None:
            _check(lib().lbm_set_solid(self._ctx, None, c_double(0.0)))
            return
        m = np.ascontiguousarray(np.asarray(solid, dtype=bool).astype(np.uint8))
        if m.shape != self.shape:
            raise ValueError(f"solid mask must have shape {self.shape}")
        _check(lib().lbm_set_solid(self._ctx, c_void_p(m.ctypes.data), c_double(float(psi_wall))))

    def _to_device(self, a, shape):
        torch = self.torch
        t = torch.as_tensor(a, dtype=torch.float64)
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"expected shape {shape}, got {tuple(t.shape)}")
        return t.to(self.workspace.device).contiguous()

    def step(self, n: int = 1):
        _check(lib().lbm_step(self._ctx, int(n)))

    def step_timed(self, n: int):
        """Run n steps with HIP events around every kernel; returns the summed
        kernel durations in ms: (psi pass or fused kernel, collide pass)."""
        ms = np.zeros(2)
        _check(lib().lbm_step_timed(self._ctx, int(n), _dptr(ms)))
        return float(ms[0]), float(ms[1])

    def check(self):
        _check(lib().lbm_check(self._ctx))

    def clear_error(self):
        _check(lib().lbm_clear_error(self._ctx))

    def set_gamma(self, gamma):
        g = np.ascontiguousarray(np.asarray(gamma, dtype=np.float64))
        if g.shape != (self.nc,):
            raise ValueError(f"gamma must have {self.nc} entries")
        _check(lib().lbm_set_gamma(self._ctx, _dptr(g)))

    def moments(self, fields=True, totals=True, noalloc=False):
        """Fields and conservation totals of the current state (lbm_moments, or
        lbm_moments_noalloc, whose partial sums use the library's static scratch)."""
        torch = self.torch
        dev = self.workspace.device
        out = {}
        ptrs = [None, None, None, None]
        if fields:
            out["rho_s"] = torch.empty((self.nc,) + self.shape, dtype=torch.float64, device=dev)
            out["u"] = torch.empty((self.D,) + self.shape, dtype=torch.float64, device=dev)
            out["p"] = torch.empty(self.shape, dtype=torch.float64, device=dev)
            out["psi"] = torch.empty(self.shape, dtype=torch.float64, device=dev)
            ptrs = [c_void_p(out[k].data_ptr()) for k in ("rho_s", "u", "p", "psi")]
        tot = np.zeros(2 * self.nc + 2 * self.D) if totals else None
        self._inputs_ready()
        fn = lib().lbm_moments_noalloc if noalloc else lib().lbm_moments
        _check(fn(self._ctx, *ptrs, None if tot is None else _dptr(tot)))
        self._outputs_ready()
        if totals:
            out["mass"] = tot[: self.nc].copy()
            out["momentum"] = tot[self.nc: self.nc + self.D].copy()
            out["force"] = tot[self.nc + self.D: self.nc + 2 * self.D].copy()
            out["negative_cells"] = tot[self.nc + 2 * self.D:].astype(np.int64)
        return out

    def get_populations(self):
        torch = self.torch
        f = torch.empty((self.nc, self.Q) + self.shape, dtype=torch.float64, device=self.workspace.device)
        self._inputs_ready()
        _check(lib().lbm_get_populations(self._ctx, c_void_p(f.data_ptr())))
        self._outputs_ready()
        return f

    def set_populations(self, f):
        t = self._to_device(f, (self.nc, self.Q) + self.shape)
        self._inputs_ready()
        _check(lib().lbm_set_populations(self._ctx, c_void_p(t.data_ptr())))
        self.stream.synchronize()

    # -- discrete adjoint ---------------------------------------------------
    def _adjoint_ws(self, nsteps, checkpoint_every):
        nbytes = c_size_t(0)
        _check(lib().lbm_adjoint_workspace(self._ctx, int(nsteps), int(checkpoint_every), ctypes.byref(nbytes)))
        ws = self.torch.empty(int(nbytes.value) + 256, dtype=self.torch.uint8, device=self.workspace.device)
        return ws, (ws.data_ptr() + 255) // 256 * 256, int(nbytes.value)

    def step_adjoint(self, h_next):
        """One reverse step at the current state: returns (dL/df(t) as a float64
        device tensor [nc, Q, *shape], dL/daa [nc, nc], dL/db [nc] through the EOS)."""
        torch = self.torch
        h = self._to_device(h_next, (self.nc, self.Q) + self.shape)
        out = torch.empty_like(h)
        daa = np.zeros(self.nc * self.nc)
        db = np.zeros(self.nc)
        ws, ptr, nbytes = self._adjoint_ws(1, 1)
        self._inputs_ready()
        _check(lib().lbm_step_adjoint(self._ctx, c_void_p(h.data_ptr()), c_void_p(out.data_ptr()), _dptr(daa),
                                      _dptr(db), c_void_p(ptr), c_size_t(nbytes)))
        self._outputs_ready()
        del ws
        return out, daa.reshape(self.nc, self.nc), db

    def adjoint(self, nsteps, checkpoint_every, mask, x_target):
        """Advance nsteps with checkpoints, then return {"loss", "x_liq", "d_k" (nc x nc),
        "d_a", "d_b"} of L = sum (x_liq - x_target)^2 over the cells where mask != 0."""
        torch = self.torch
        m = torch.as_tensor(np.asarray(mask), dtype=torch.uint8)
        if tuple(m.shape) != self.shape:
            raise ValueError(f"mask must have shape {self.shape}")
        m = m.to(self.workspace.device).contiguous()
        xt = np.ascontiguousarray(np.asarray(x_target, dtype=np.float64))
        if xt.shape != (self.nc,):
            raise ValueError(f"x_target must have {self.nc} entries")
        loss = np.zeros(1)
        x = np.zeros(self.nc)
        dk = np.zeros(self.nc * self.nc)
        da = np.zeros(self.nc)
        db = np.zeros(self.nc)
        ws, ptr, nbytes = self._adjoint_ws(nsteps, checkpoint_every)
        self._inputs_ready()
        _check(lib().lbm_adjoint(self._ctx, int(nsteps), int(checkpoint_every), c_void_p(m.data_ptr()), _dptr(xt),
                                 c_void_p(ptr), c_size_t(nbytes), _dptr(loss), _dptr(x), _dptr(dk), _dptr(da),
                                 _dptr(db)))
        del ws
        return {"loss": float(loss[0]), "x_liq": x, "d_k": dk.reshape(self.nc, self.nc), "d_a": da, "d_b": db}

    def close(self):
        if getattr(self, "_ctx", None) is not None:
            if self._own_stream:
                self.stream.synchronize()      # the workspace goes back to torch
            lib().lbm_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def eos_param_grad(mix: dict, T: float, d_aa, d_b_direct):
    """Chain EOS-table derivatives to (d_k [nc, nc], d_a [nc], d_b [nc]) (host)."""
    m = mixture_struct(mix)
    nc = m.nc
    daa = np.ascontiguousarray(np.asarray(d_aa, dtype=np.float64).reshape(nc * nc))
    dbd = np.ascontiguousarray(np.asarray(d_b_direct, dtype=np.float64).reshape(nc))
    dk = np.zeros(nc * nc)
    da = np.zeros(nc)
    db = np.zeros(nc)
    _check(lib().lbm_eos_param_grad(ctypes.byref(m), float(T), _dptr(daa), _dptr(dbd), _dptr(dk), _dptr(da),
                                    _dptr(db)))
    return dk.reshape(nc, nc), da, db


class LbmBatch:
    """Many independent boxes advanced together (one lbm_batch).

    boxes: list of dicts {"mix", "shape" (ny, nx) or (nz, ny, nx), "T", "tau", "beta",
    "gamma", "rho0" (nc, *shape)}, optionally "solid" (*shape, bool) and "psi_wall"
    for walls (the model of lbm_set_solid).  With graph_steps > 0 the batch runs on
    its own (default-priority) stream so the steps can be captured in a HIP graph.
    fused=True runs one launch per step (D2Q9 with "f32" / "f16" storage only; see
    lbm_batch_params.fused).
    """

    def __init__(self, boxes, lattice="D2Q9", collision="bgk", forcing="edm", storage="f64", tile=0,
                 graph_steps=0, grid=0, mrt_s=None, accel=None, G=-1.0, device="cuda", fused=False):
        import torch
        self.torch = torch
        self.lattice = lattice
        self.Q = Q_OF[lattice]
        n = len(boxes)
        arr = (LbmBox * n)()
        self.shapes, self.ncs = [], []
        masks = []                         # alive until lbm_batch_init has read them
        for i, bx in enumerate(boxes):
            shape = tuple(int(v) for v in bx["shape"])
            if lattice == "D2Q9":
                ny, nx = shape
                nz = 1
            else:
                nz, ny, nx = shape
            arr[i].mix = mixture_struct(bx["mix"])
            arr[i].nx, arr[i].ny, arr[i].nz = nx, ny, nz
            arr[i].T = float(bx["T"])
            arr[i].tau = float(bx.get("tau", 0.8))
            arr[i].G = float(bx.get("G", G))
            arr[i].beta = float(bx["beta"])
            for k, g in enumerate(bx["gamma"]):
                arr[i].gamma[k] = float(g)
            if bx.get("solid") is not None:
                m = np.ascontiguousarray(np.asarray(bx["solid"], dtype=bool).astype(np.uint8))
                if m.shape != shape:
                    raise ValueError(f"box {i}: solid mask must have shape {shape}")
                masks.append(m)
                arr[i].solid = m.ctypes.data
                arr[i].psi_wall = float(bx.get("psi_wall", 0.0))
            nc_b = len(bx["mix"]["a"])
            if tuple(np.shape(bx["rho0"])) != (nc_b,) + shape:
                raise ValueError(f"box {i}: rho0 must have shape {(nc_b,) + shape}, got {tuple(np.shape(bx['rho0']))}")
            self.shapes.append(shape)
            self.ncs.append(nc_b)
        self._boxes = arr
        prm = LbmBatchParams()
        prm.lattice = LATTICES[lattice]
        prm.collision = COLLISIONS[collision]
        prm.forcing = FORCINGS[forcing]
        prm.storage = STORAGES[storage]
        prm.tile = int(tile)
        prm.graph_steps = int(graph_steps)
        prm.grid = int(grid)
        prm.fused = 1 if fused else 0
        if mrt_s is not None:
            for k, v in enumerate(mrt_s):
                prm.mrt_s[k] = float(v)
        if accel is not None:
            for d, v in enumerate(accel):
                prm.accel[d] = float(v)
        self._prm = prm
        ws, fe, pe = c_size_t(0), c_size_t(0), c_size_t(0)
        _check(lib().lbm_batch_layout(arr, n, ctypes.byref(prm), ctypes.byref(ws), ctypes.byref(fe),
                                      ctypes.byref(pe)))
        self.field_elems, self.pop_elems = int(fe.value), int(pe.value)
        self.stream = torch.cuda.Stream(device=device) if graph_steps > 0 else torch.cuda.current_stream(device)
        cur = torch.cuda.current_stream(device)
        self.workspace = torch.empty(int(ws.value) + 256, dtype=torch.uint8, device=device)
        wsp = (self.workspace.data_ptr() + 255) // 256 * 256
        rho0 = torch.cat([torch.as_tensor(bx["rho0"], dtype=torch.float64).reshape(-1) for bx in boxes]).to(device)
        if rho0.numel() != self.field_elems:
            raise ValueError(f"initial fields hold {rho0.numel()} values, the batch layout {self.field_elems}")
        self.stream.wait_stream(cur)
        ctx = c_void_p()
        _check(lib().lbm_batch_init(arr, n, ctypes.byref(prm), c_void_p(wsp), c_size_t(int(ws.value)),
                                    c_void_p(rho0.data_ptr()), c_void_p(self.stream.cuda_stream),
                                    ctypes.byref(ctx)))
        del masks
        self._ctx = ctx

    def step(self, n=1):
        _check(lib().lbm_batch_step(self._ctx, int(n)))

    def check(self):
        _check(lib().lbm_batch_check(self._ctx))

    def set_gamma(self, box, gamma):
        g = np.ascontiguousarray(np.asarray(gamma, dtype=np.float64))
        _check(lib().lbm_batch_set_gamma(self._ctx, int(box), _dptr(g)))

    def box_errors(self):
        """Per-box error flags (numpy int array, 1 = the box left the EOS domain)."""
        flags = (c_int * len(self.shapes))()
        _check(lib().lbm_batch_box_errors(self._ctx, flags))
        return np.array(flags[:], dtype=np.int64)

    def fields(self, populations=False):
        """Per-box rbar (list of (nc, *shape) tensors) and optionally populations."""
        torch = self.torch
        dev = self.workspace.device
        rho = torch.empty(self.field_elems, dtype=torch.float64, device=dev)
        f = torch.empty(self.pop_elems, dtype=torch.float64, device=dev) if populations else None
        self.stream.wait_stream(torch.cuda.current_stream(dev))
        _check(lib().lbm_batch_fields(self._ctx, c_void_p(rho.data_ptr()),
                                      None if f is None else c_void_p(f.data_ptr())))
        self.stream.synchronize()
        out_r, out_f = [], []
        o, of = 0, 0
        for shape, nc in zip(self.shapes, self.ncs):
            cells = int(np.prod(shape))
            out_r.append(rho[o: o + nc * cells].reshape((nc,) + shape))
            o += nc * cells
            if f is not None:
                out_f.append(f[of: of + nc * self.Q * cells].reshape((nc, self.Q) + shape))
                of += nc * self.Q * cells
        return (out_r, out_f) if populations else out_r

    def close(self):
        if getattr(self, "_ctx", None) is not None:
            lib().lbm_batch_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
