"""ctypes binding of the C ABI in ``include/tlb.h`` (argument marshalling only).

Every step of the lattice Boltzmann update runs in the HIP library
``lib/libtlb.so``; this module converts numpy arrays to the plain pointers the
ABI takes and turns return codes into exceptions. It never computes any part
of the method and there is no fallback: if the library is missing, loading
fails with an error.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libtlb.so")

TLB_OK, TLB_EINVAL, TLB_ENOMEM, TLB_EDEVICE, TLB_ENUMERIC, TLB_ESTATE = 0, -1, -2, -3, -4, -5
PRECISIONS = {"fp64": 0, "fp32": 1, "fp16dev": 2, "bf16dev": 3, "fix16dev": 4}

# Every symbol the header declares (checked by the CPU test suite).
EXPORTS = (
    "tlb_init", "tlb_init_external", "tlb_workspace_bytes", "tlb_step", "tlb_observables",
    "tlb_get_fields", "tlb_get_stress",
    "tlb_row_averages", "tlb_droplets", "tlb_droplets_noalloc", "tlb_get_populations",
    "tlb_set_bottom_temperature", "tlb_forward_taped", "tlb_adjoint_step", "tlb_time", "tlb_launch_info", "tlb_destroy",
    "tlb_last_error",
)


class TlbError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"[{code}] {message}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [
        ("lx", ctypes.c_int32), ("ly", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("launch_flags", ctypes.c_int32),
        ("tau", ctypes.c_double), ("tau_g", ctypes.c_double),
        ("rho0", ctypes.c_double), ("g12", ctypes.c_double),
        ("g_a", ctypes.c_double * 2), ("g_r", ctypes.c_double * 2),
        ("alpha_g", ctypes.c_double), ("t_top", ctypes.c_double),
        ("rho_wall", ctypes.c_double * 2), ("dt_nominal", ctypes.c_double),
        ("rho_ref", ctypes.c_double * 2), ("t_ref", ctypes.c_double),
        ("u_wall", ctypes.c_double * 2),
        ("fused", ctypes.c_int32), ("fused_rows", ctypes.c_int32),
        ("fused_strip", ctypes.c_int32), ("rows", ctypes.c_int32), ("fused_lanes", ctypes.c_int32),
    ]


TLB_LAUNCH_GENERAL_PATH, TLB_LAUNCH_WIDE_OFFSETS = 1, 2
FUSED_MODES = {"auto": 0, "never": 1, "always": 2}
LAUNCH_KEYS = ("fused", "fused_rows", "fused_strip", "fused_lanes", "rows", "general_path",
               "wide_offsets")


class Obs(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("mass_a", ctypes.c_double), ("mass_b", ctypes.c_double),
                ("sum_t", ctypes.c_double), ("nu", ctypes.c_double), ("nu_top", ctypes.c_double),
                ("ke", ctypes.c_double)]


class Launch(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int32) for k in
                ("bx", "rows", "grid_x", "grid_y",
                 "fused_rows", "fused_strip", "fused_grid_x", "fused_grid_y", "fused_lanes")]


class Droplet(ctypes.Structure):
    _fields_ = [("root", ctypes.c_int64), ("size", ctypes.c_int64), ("mass", ctypes.c_double),
                ("x", ctypes.c_double), ("y", ctypes.c_double), ("nu", ctypes.c_double)]


# the same record as a numpy structured type (filled by the library in place)
DROPLET_DTYPE = np.dtype([(k, np.int64 if k in ("root", "size") else np.float64)
                          for k, _ in Droplet._fields_], align=True)
assert DROPLET_DTYPE.itemsize == ctypes.sizeof(Droplet)


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load ``libtlb.so``; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(
            f"HIP library not built: {path} is missing (run `python -m paper_2109_12565_amd.build`)")
    # torch ships its own HIP runtime and opens it under a file name that does
    # not match the SONAME of the system copy this library links; loading
    # torch first makes both resolve to torch's copy, so the process holds a
    # single HIP runtime and torch's streams are valid handles here.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    vp = ctypes.c_void_p
    lib.tlb_init.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(Params), dp, dp, dp, dp, dp,
                             ctypes.POINTER(ctypes.c_uint8), dp, vp]
    lib.tlb_init_external.argtypes = lib.tlb_init.argtypes + [vp, ctypes.c_int64]
    lib.tlb_workspace_bytes.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_uint8)]
    lib.tlb_workspace_bytes.restype = ctypes.c_int64
    lib.tlb_step.argtypes = [vp, ctypes.c_int64]
    lib.tlb_observables.argtypes = [vp, ctypes.POINTER(Obs)]
    lib.tlb_get_fields.argtypes = [vp, dp, dp, dp, dp, dp]
    lib.tlb_get_populations.argtypes = [vp, dp]
    lib.tlb_get_stress.argtypes = [vp, dp, dp]
    lib.tlb_row_averages.argtypes = [vp, dp, dp]
    for name in ("tlb_droplets", "tlb_droplets_noalloc"):
        getattr(lib, name).argtypes = [vp, ctypes.c_double, vp, ctypes.c_int64,
                                       ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32)]
    lib.tlb_set_bottom_temperature.argtypes = [vp, dp]
    lib.tlb_forward_taped.argtypes = [vp, ctypes.c_int64, ctypes.c_int32, dp]
    lib.tlb_adjoint_step.argtypes = [vp, ctypes.c_int64, ctypes.c_double, dp]
    lib.tlb_time.argtypes = [vp]
    lib.tlb_time.restype = ctypes.c_int64
    lib.tlb_launch_info.argtypes = [vp, ctypes.POINTER(Launch)]
    lib.tlb_destroy.argtypes = [vp]
    lib.tlb_last_error.argtypes = [vp]
    lib.tlb_last_error.restype = ctypes.c_char_p
    for name in ("tlb_init", "tlb_init_external", "tlb_step", "tlb_observables",
                 "tlb_get_fields", "tlb_get_stress",
                 "tlb_row_averages", "tlb_droplets", "tlb_droplets_noalloc",
                 "tlb_get_populations", "tlb_set_bottom_temperature",
                 "tlb_forward_taped", "tlb_adjoint_step", "tlb_launch_info", "tlb_destroy"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _dp(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _field(a, shape, name):
    if a is None:
        return None
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if a.shape != shape:
        raise ValueError(f"{name}: expected shape {shape}, got {a.shape}")
    return a


def _current_stream():
    """torch's current HIP stream on the current device, or None."""
    try:
        import torch
    except ImportError:
        return None
    if not torch.cuda.is_available():
        return None
    return torch.cuda.current_stream().cuda_stream


class Simulation:
    """A lattice state on the GPU behind one ``tlb_handle``.

    ``params`` holds the model constants named as in ``tlb_params`` (tau,
    tau_g, rho0, g12, g_a, g_r, alpha_g, t_top, rho_wall, dt_nominal, and
    optionally rho_ref, t_ref for the 16-bit storages: by default rho0 for
    both components and the mean of the two wall temperatures; u_wall, the
    x-velocities of the bottom and top walls, by default at rest).
    Field arrays are (ly, lx) with x fastest. By default the work runs on
    torch's current stream.

    ``device_memory``: "library" (the library allocates its device buffers)
    or "torch" (the state and step buffers live in a uint8 tensor that
    torch's caching allocator owns, through ``tlb_init_external``).

    ``launch`` (optional) sets the launch choices of ``tlb_params``: ``fused``
    ("auto", "never", "always"), ``fused_rows``, ``fused_strip``, ``fused_lanes``, ``rows``
    (0 or absent: chosen by the library), and the kernel-selection flags
    ``general_path`` and ``wide_offsets``.
    """

    def __init__(self, params: dict, rho_a, rho_b, temp, *, solid=None, t_bottom=None,
                 ux0=None, uy0=None, precision: str = "fp32", stream="torch", launch=None,
                 device_memory: str = "library"):
        self._lib = load_library()
        self._h = ctypes.c_void_p()
        rho_a = np.ascontiguousarray(np.asarray(rho_a, dtype=np.float64))
        if rho_a.ndim != 2:
            raise ValueError("rho_a must be 2-D (ly, lx)")
        ly, lx = rho_a.shape
        self.shape = (ly, lx)
        rho_b = _field(rho_b, self.shape, "rho_b")
        temp = _field(temp, self.shape, "temp")
        ux0 = _field(ux0, self.shape, "ux0")
        uy0 = _field(uy0, self.shape, "uy0")
        if (ux0 is None) != (uy0 is None):
            raise ValueError("give both ux0 and uy0 or neither")
        sol = None
        if solid is not None:
            sol = np.ascontiguousarray(np.asarray(solid, dtype=np.uint8))
            if sol.shape != self.shape:
                raise ValueError(f"solid: expected shape {self.shape}, got {sol.shape}")
        if t_bottom is None:
            t_bottom = 1.0
        t_bottom = np.ascontiguousarray(np.broadcast_to(np.asarray(t_bottom, np.float64), (lx,)))
        if precision not in PRECISIONS:
            raise ValueError(f"precision must be one of {sorted(PRECISIONS)}")
        launch = dict(launch or {})
        unknown = set(launch) - set(LAUNCH_KEYS)
        if unknown:
            raise ValueError(f"unknown launch options {sorted(unknown)}")
        p = Params()
        p.lx, p.ly, p.precision = lx, ly, PRECISIONS[precision]
        p.launch_flags = ((TLB_LAUNCH_GENERAL_PATH if launch.get("general_path") else 0) |
                          (TLB_LAUNCH_WIDE_OFFSETS if launch.get("wide_offsets") else 0))
        p.fused = FUSED_MODES[launch.get("fused", "auto")]
        p.fused_rows = int(launch.get("fused_rows", 0))
        p.fused_strip = int(launch.get("fused_strip", 0))
        p.rows = int(launch.get("rows", 0))
        p.fused_lanes = int(launch.get("fused_lanes", 0))
        p.tau, p.tau_g = params["tau"], params["tau_g"]
        p.rho0, p.g12 = params["rho0"], params["g12"]
        p.g_a[0], p.g_a[1] = params["g_a"]
        p.g_r[0], p.g_r[1] = params["g_r"]
        p.alpha_g, p.t_top = params["alpha_g"], params["t_top"]
        p.rho_wall[0], p.rho_wall[1] = params["rho_wall"]
        p.dt_nominal = params["dt_nominal"]
        rr = params.get("rho_ref", (params["rho0"], params["rho0"]))
        p.rho_ref[0], p.rho_ref[1] = rr
        p.t_ref = params.get("t_ref", 0.5 * (float(np.mean(t_bottom)) + params["t_top"]))
        p.u_wall[0], p.u_wall[1] = params.get("u_wall", (0.0, 0.0))
        self.params = p
        self.precision = precision
        # droplet records asked for by droplets(): room for one droplet per
        # 64 nodes (emulsions of radius-10 discs hold one per ~600), raised
        # to the count when a call finds more
        self._drop_cap = max(4096, lx * ly // 64)
        self._tape_generation = 0  # bumped by every forward_taped
        s = _current_stream() if stream == "torch" else stream
        sol_p = None if sol is None else sol.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        args = (ctypes.byref(self._h), ctypes.byref(p), _dp(rho_a), _dp(rho_b), _dp(temp),
                _dp(ux0), _dp(uy0), sol_p, _dp(t_bottom), ctypes.c_void_p(s) if s else None)
        if device_memory not in ("library", "torch"):
            raise ValueError("device_memory must be 'library' or 'torch'")
        self._workspace = None
        if device_memory == "torch":
            # the step path's buffers in a tensor torch's allocator owns
            import torch
            nbytes = self._lib.tlb_workspace_bytes(ctypes.byref(p), sol_p)
            if nbytes < 0:
                raise TlbError(int(nbytes), self._lib.tlb_last_error(None).decode())
            self._workspace = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
            rc = self._lib.tlb_init_external(*args, ctypes.c_void_p(self._workspace.data_ptr()),
                                             int(nbytes))
        else:
            rc = self._lib.tlb_init(*args)
        if rc != TLB_OK:
            raise TlbError(rc, self._lib.tlb_last_error(None).decode())

    def _check(self, rc):
        if rc != TLB_OK:
            raise TlbError(rc, self._lib.tlb_last_error(self._h).decode())

    @property
    def t(self) -> int:
        return int(self._lib.tlb_time(self._h))

    def launch_info(self) -> dict:
        """Launch geometry of the step kernels (fused_rows > 0: the fused
        two-step kernel advances pairs of steps)."""
        g = Launch()
        self._check(self._lib.tlb_launch_info(self._h, ctypes.byref(g)))
        return {k: getattr(g, k) for k, _ in Launch._fields_}

    def step(self, n: int = 1) -> "Simulation":
        self._check(self._lib.tlb_step(self._h, int(n)))
        return self

    def observables(self) -> dict:
        o = Obs()
        self._check(self._lib.tlb_observables(self._h, ctypes.byref(o)))
        return {k: getattr(o, k) for k, _ in Obs._fields_}

    def fields(self) -> dict:
        ly, lx = self.shape
        out = {k: np.empty((ly, lx)) for k in ("rho_a", "rho_b", "ux", "uy", "temp")}
        self._check(self._lib.tlb_get_fields(self._h, *(_dp(out[k]) for k in
                                                       ("rho_a", "rho_b", "ux", "uy", "temp"))))
        return out

    def stress(self) -> dict:
        """xy stress of the current time, (ly, lx) each: the viscous part
        ``sxy_visc`` and the interaction pressure tensor ``pxy_int`` (the
        total stress is their difference)."""
        ly, lx = self.shape
        out = {k: np.empty((ly, lx)) for k in ("sxy_visc", "pxy_int")}
        self._check(self._lib.tlb_get_stress(self._h, _dp(out["sxy_visc"]), _dp(out["pxy_int"])))
        return out

    def row_averages(self) -> dict:
        """Fluid-node means of u^H_x and of the total xy stress per row, (ly,)."""
        ly = self.shape[0]
        out = {"u_av": np.empty(ly), "pxy_av": np.empty(ly)}
        self._check(self._lib.tlb_row_averages(self._h, _dp(out["u_av"]), _dp(out["pxy_av"])))
        return out

    def droplets(self, threshold: float = 0.8, labels: bool = False, noalloc: bool = False) -> dict:
        """Droplets of the current time: arrays root, size, mass, x, y, nu
        (numbered by smallest node index) and, if asked, the node labels
        (ly, lx) with -1 outside droplets. ``noalloc`` calls
        ``tlb_droplets_noalloc`` (static device workspace, no allocation)."""
        ly, lx = self.shape
        count = ctypes.c_int64()
        lab = np.empty((ly, lx), np.int32) if labels else None
        lab_p = lab.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) if labels else None
        fn = self._lib.tlb_droplets_noalloc if noalloc else self._lib.tlb_droplets
        arr = self._droplet_records()
        self._check(fn(self._h, float(threshold), arr.ctypes.data, len(arr), ctypes.byref(count),
                       lab_p))
        n = count.value
        if n > len(arr):  # more droplets than room: ask again with room for all
            self._drop_cap = n
            arr = self._droplet_records()
            self._check(fn(self._h, float(threshold), arr.ctypes.data, n, ctypes.byref(count),
                           None))
        out = {k: np.ascontiguousarray(arr[k][:n]) for k in DROPLET_DTYPE.names}
        if labels:
            out["label"] = lab
        return out

    def _droplet_records(self) -> np.ndarray:
        """Room for ``_drop_cap`` droplet records, in page-locked host memory
        (the copy from the device is then one DMA, with no staging), kept
        for the next call."""
        buf = getattr(self, "_drop_buf", None)
        if buf is None or len(buf) < self._drop_cap:
            import torch
            raw = torch.empty(self._drop_cap * DROPLET_DTYPE.itemsize, dtype=torch.uint8,
                              pin_memory=True)
            buf = np.frombuffer(raw.numpy(), DROPLET_DTYPE)
            self._drop_raw, self._drop_buf = raw, buf
        return buf

    def populations(self) -> np.ndarray:
        """Post-collision f*_A, f*_B, g* of the current time, [27, ly, lx]."""
        ly, lx = self.shape
        out = np.empty((27, ly, lx))
        self._check(self._lib.tlb_get_populations(self._h, _dp(out)))
        return out

    def set_bottom_temperature(self, t_bottom) -> None:
        tb = np.ascontiguousarray(np.broadcast_to(np.asarray(t_bottom, np.float64), (self.shape[1],)))
        self._check(self._lib.tlb_set_bottom_temperature(self._h, _dp(tb)))

    def forward_taped(self, nsteps: int, ckpt_every: int = 25) -> float:
        """Advance ``nsteps`` steps keeping checkpoints every ``ckpt_every``
        (0: chosen by the library from the free device memory); returns the
        time-averaged top-wall Nusselt number over them."""
        loss = ctypes.c_double()
        self._tape_generation += 1
        self._check(self._lib.tlb_forward_taped(self._h, int(nsteps), int(ckpt_every),
                                                ctypes.byref(loss)))
        return loss.value

    @property
    def tape_generation(self) -> int:
        """Number of taped runs started on this handle (identifies the tape
        that a later ``adjoint`` call sweeps)."""
        return self._tape_generation

    def adjoint(self, nsteps: int, seed: float = 1.0) -> np.ndarray:
        """``seed`` times the gradient of the taped loss with respect to the
        bottom wall temperature, shape (lx,)."""
        out = np.empty(self.shape[1])
        self._check(self._lib.tlb_adjoint_step(self._h, int(nsteps), float(seed), _dp(out)))
        return out

    def close(self) -> None:
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.tlb_destroy(h)  # synchronises the stream first
            self._h = ctypes.c_void_p()
        self._workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def _autograd_function():
    import torch

    class TopNusseltLoss(torch.autograd.Function):
        """L(T_b) = time-averaged top-wall Nusselt number of ``nsteps`` steps of
        ``sim`` from its current state, differentiable in the bottom wall
        temperature ``t_bottom`` (an (lx,) tensor) through the library's
        discrete adjoint. The forward call advances ``sim``."""

        @staticmethod
        def forward(ctx, t_bottom, sim, nsteps, ckpt_every):
            sim.set_bottom_temperature(t_bottom.detach().to("cpu", torch.float64).numpy())
            loss = sim.forward_taped(nsteps, ckpt_every)
            ctx.sim, ctx.nsteps = sim, nsteps
            ctx.generation = sim.tape_generation
            ctx.dtype, ctx.device = t_bottom.dtype, t_bottom.device
            return torch.tensor(loss, dtype=t_bottom.dtype, device=t_bottom.device)

        @staticmethod
        def backward(ctx, grad_out):
            if ctx.sim.tape_generation != ctx.generation:
                # the handle holds one tape: a later taped run replaced it
                raise RuntimeError(
                    "top_nusselt_loss: the simulation was taped again after this loss was "
                    "formed; its tape is gone (differentiate each loss before the next taped "
                    "run on the same Simulation)")
            g = ctx.sim.adjoint(ctx.nsteps, float(grad_out))
            return torch.as_tensor(g, dtype=ctx.dtype).to(ctx.device), None, None, None

    return TopNusseltLoss


def top_nusselt_loss(sim: Simulation, t_bottom, nsteps: int, ckpt_every: int = 25):
    """Differentiable time-averaged top-wall Nusselt number (see
    ``TopNusseltLoss``)."""
    return _autograd_function().apply(t_bottom, sim, nsteps, ckpt_every)
