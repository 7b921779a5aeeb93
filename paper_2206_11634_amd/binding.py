"""ctypes binding of libmdlbm (include/mdlbm.h).

Argument marshalling only: every step of the lattice update runs in the HIP
library.  Device memory comes from PyTorch (ROCm build) and work is enqueued
on torch's current stream.  Loading fails loudly when the library has not been
built or no GPU is present; there is no CPU fallback.

Module-level functions carry the C-ABI names (lbm_init, lbm_classify_nodes,
lbm_step, lbm_particle_forces, dem_step, ...); the `Lattice` and
`DeviceParticles` classes hold the buffers those calls need.
"""
from __future__ import annotations

import ctypes
from pathlib import Path

import numpy as np

LIB_PATH = Path(__file__).resolve().parent / "libmdlbm.so"
Q = 19

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_ECAPACITY, LBM_ENUMERIC, LBM_EDEVICE, LBM_ESTATE = range(7)
STORAGE = {"f64": 0, "f32": 1, "f16": 2}
TREAT_VIBB, TREAT_MISSING, TREAT_EXACT_Q, TREAT_NEQ_SPLIT = 1, 2, 4, 8
LINK_VIBB, LINK_HALFWAY, LINK_MISSING = 0, 1, 2
FORCE_SUM_ATOMIC, FORCE_SUM_EXACT = 0, 1

_P = ctypes.c_void_p


class LbmConfig(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("periodic", ctypes.c_int32 * 3), ("tau", ctypes.c_double),
                ("rho0", ctypes.c_double), ("u0", ctypes.c_double * 3),
                ("body_force", ctypes.c_double * 3), ("storage", ctypes.c_int32),
                ("treatments", ctypes.c_int32), ("n_particles", ctypes.c_int32),
                ("n_ctrl", ctypes.c_int32), ("box_half", ctypes.c_int32),
                ("h16_scale", ctypes.c_double), ("stream", _P), ("classify_mode", ctypes.c_int32),
                ("lattice", ctypes.c_int32), ("force_sum", ctypes.c_int32)]


class LbmSizes(ctypes.Structure):
    _fields_ = [("ncell", ctypes.c_int64), ("cell_stride", ctypes.c_int64),
                ("population_bytes", ctypes.c_size_t), ("owner_bytes", ctypes.c_size_t),
                ("flag_bytes", ctypes.c_size_t), ("moment_bytes", ctypes.c_size_t),
                ("checkpoint_bytes", ctypes.c_size_t), ("adjoint_bytes", ctypes.c_size_t),
                ("dem_checkpoint_bytes", ctypes.c_size_t),
                ("contact_adjoint_bytes", ctypes.c_size_t)]


class LbmBuffers(ctypes.Structure):
    _fields_ = [("f_dev", _P * 2), ("owner_dev", _P * 2), ("flag_dev", _P), ("moments_dev", _P)]


class LbmParticles(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("ctrl_off", _P), ("body_pts", _P), ("K", _P),
                ("c0", _P), ("rs", _P), ("mass", _P), ("volume", _P), ("inertia", _P),
                ("pos", _P), ("quat", _P), ("vel", _P), ("omega", _P), ("world_pts", _P)]


class LbmCounts(ctypes.Structure):
    _fields_ = [("n_links", ctypes.c_int64), ("n_refill", ctypes.c_int64),
                ("n_candidates", ctypes.c_int64)]


class DemParams(ctypes.Structure):
    _fields_ = [("kn", ctypes.c_double), ("eta_n", ctypes.c_double), ("kt", ctypes.c_double),
                ("eta_t", ctypes.c_double), ("mu_s", ctypes.c_double), ("ctol", ctypes.c_double),
                ("newton_tol", ctypes.c_double), ("newton_iter", ctypes.c_int32),
                ("gravity", ctypes.c_double * 3), ("rho_f", ctypes.c_double)]

    @classmethod
    def make(cls, kn=0.0, eta_n=0.0, kt=0.0, eta_t=0.0, mu_s=0.3, ctol=1e-3, newton_tol=1e-12,
             newton_iter=50, gravity=(0.0, 0.0, 0.0), rho_f=1.0):
        return cls(kn, eta_n, kt, eta_t, mu_s, ctol, newton_tol, newton_iter,
                   (ctypes.c_double * 3)(*gravity), rho_f)


class LbmProfile(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 8), ("launches", ctypes.c_int64 * 8)]


CLASSIFY = {"auto": 0, "sweep": 1, "balls": 2}

PHASES = ("bulk", "boundary", "classify", "refill", "dem", "adjoint")

EXPORTS = ["lbm_query_sizes", "lbm_init", "lbm_destroy", "lbm_last_error", "lbm_classify_nodes",
           "lbm_classify_nodes_async",
           "lbm_step", "lbm_particle_forces", "dem_step", "lbm_get_links", "lbm_get_refill",
           "lbm_get_owner", "lbm_get_populations", "lbm_set_populations", "lbm_synchronize",
           "lbm_profile_enable", "lbm_profile_read", "lbm_checkpoint_save", "lbm_checkpoint_load",
           "lbm_tape_begin", "lbm_adjoint", "lbm_adjoint_coupled", "lbm_get_moments",
           "lbm_dem_checkpoint_save", "lbm_dem_checkpoint_load", "dem_step_noalloc",
           "lbm_geometry_bytes", "lbm_geometry_save", "lbm_geometry_load", "lbm_step_dem"]

_lib = None


def load(path: Path | None = None):
    """Load the built library (no compute).  Raises when it is missing."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = Path(path) if path else LIB_PATH
    if not p.exists():
        raise RuntimeError(f"{p} is not built; run `python -m paper_2206_11634_amd.build` "
                           "(the lattice update has no CPU fallback)")
    # torch first: its HIP runtime must be the one the library binds to
    import torch  # noqa: F401
    L = ctypes.CDLL(str(p))
    sig = {
        "lbm_query_sizes": [ctypes.POINTER(LbmConfig), ctypes.POINTER(LbmSizes)],
        "lbm_init": [ctypes.POINTER(LbmConfig), ctypes.POINTER(LbmBuffers), ctypes.POINTER(_P)],
        "lbm_destroy": [_P],
        "lbm_classify_nodes": [_P, ctypes.POINTER(LbmParticles), ctypes.POINTER(LbmCounts)],
        "lbm_classify_nodes_async": [_P, ctypes.POINTER(LbmParticles)],
        "lbm_step": [_P, ctypes.POINTER(LbmParticles)],
        "lbm_particle_forces": [_P, _P, _P],
        "dem_step": [_P, ctypes.POINTER(LbmParticles), ctypes.c_int, ctypes.c_double,
                     ctypes.POINTER(DemParams)],
        "dem_step_noalloc": [_P, ctypes.POINTER(LbmParticles), ctypes.c_int, ctypes.c_double,
                             ctypes.POINTER(DemParams)],
        "lbm_step_dem": [_P, ctypes.POINTER(LbmParticles), ctypes.c_int, ctypes.c_double,
                         ctypes.POINTER(DemParams)],
        "lbm_get_links": [_P, ctypes.c_int64, _P, _P, _P, _P, _P, ctypes.POINTER(ctypes.c_int64)],
        "lbm_get_refill": [_P, ctypes.c_int64, _P, _P, ctypes.POINTER(ctypes.c_int64)],
        "lbm_get_owner": [_P, _P],
        "lbm_get_populations": [_P, _P],
        "lbm_set_populations": [_P, _P],
        "lbm_synchronize": [_P],
        "lbm_profile_enable": [_P, ctypes.c_int],
        "lbm_profile_read": [_P, ctypes.POINTER(LbmProfile)],
        "lbm_checkpoint_save": [_P, _P],
        "lbm_checkpoint_load": [_P, _P],
        "lbm_tape_begin": [_P, ctypes.c_int],
        "lbm_get_moments": [_P, _P, _P],
        "lbm_dem_checkpoint_save": [_P, _P],
        "lbm_dem_checkpoint_load": [_P, _P],
        "lbm_geometry_bytes": [_P, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_uint64)],
        "lbm_geometry_save": [_P, _P],
        "lbm_geometry_load": [_P, _P, ctypes.c_uint64, ctypes.POINTER(LbmParticles)],
        "lbm_adjoint": [_P, ctypes.POINTER(LbmParticles), _P, _P, _P, _P],
        "lbm_adjoint_coupled": [_P, ctypes.POINTER(LbmParticles), _P, ctypes.POINTER(DemParams),
                                ctypes.c_int, ctypes.c_double, _P, _P, _P, _P],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    L.lbm_last_error.argtypes = [_P]
    L.lbm_last_error.restype = ctypes.c_char_p
    if path is None:
        _lib = L
    return L


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libmdlbm status {code}: {msg}")
        self.code = code


def _check(rc, ctx=None):
    if rc != LBM_OK:
        msg = load().lbm_last_error(ctx)
        raise LbmError(rc, msg.decode() if msg else "")


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("libmdlbm needs a ROCm GPU; torch.cuda.is_available() is False")
    return torch


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


# ---- C-ABI wrappers (same names) -------------------------------------------

def lbm_query_sizes(cfg: LbmConfig) -> LbmSizes:
    out = LbmSizes()
    _check(load().lbm_query_sizes(ctypes.byref(cfg), ctypes.byref(out)))
    return out


def lbm_init(cfg: LbmConfig, bufs: LbmBuffers):
    ctx = _P()
    _check(load().lbm_init(ctypes.byref(cfg), ctypes.byref(bufs), ctypes.byref(ctx)))
    return ctx


def lbm_destroy(ctx):
    _check(load().lbm_destroy(ctx))


def lbm_classify_nodes(ctx, parts: LbmParticles) -> LbmCounts:
    out = LbmCounts()
    _check(load().lbm_classify_nodes(ctx, ctypes.byref(parts), ctypes.byref(out)), ctx)
    return out


def lbm_classify_nodes_async(ctx, parts: LbmParticles):
    _check(load().lbm_classify_nodes_async(ctx, ctypes.byref(parts)), ctx)


def lbm_step(ctx, parts: LbmParticles):
    _check(load().lbm_step(ctx, ctypes.byref(parts)), ctx)


def lbm_particle_forces(ctx, F, T):
    _check(load().lbm_particle_forces(ctx, _ptr(F), _ptr(T)), ctx)


def dem_step(ctx, parts: LbmParticles, n_sub: int, dt: float, prm: DemParams):
    _check(load().dem_step(ctx, ctypes.byref(parts), int(n_sub), float(dt), ctypes.byref(prm)),
           ctx)


def dem_step_noalloc(ctx, parts: LbmParticles, n_sub: int, dt: float, prm: DemParams):
    _check(load().dem_step_noalloc(ctx, ctypes.byref(parts), int(n_sub), float(dt),
                                   ctypes.byref(prm)), ctx)


def lbm_step_dem(ctx, parts: LbmParticles, n_sub: int, dt: float, prm: DemParams):
    _check(load().lbm_step_dem(ctx, ctypes.byref(parts), int(n_sub), float(dt),
                               ctypes.byref(prm)), ctx)


def lbm_synchronize(ctx):
    _check(load().lbm_synchronize(ctx), ctx)


# ---- buffers -----------------------------------------------------------------

class DeviceParticles:
    """FP64 device copies of a particle set, in the layout of lbm_particles."""

    FIELDS = ("body_pts", "K", "c0", "rs", "mass", "volume", "inertia", "pos", "quat", "vel",
              "omega", "world_pts")

    def __init__(self, ps, device="cuda"):
        torch = _torch()
        self.n = ps.n
        self.device = device
        self.t = {"ctrl_off": torch.as_tensor(np.ascontiguousarray(ps.ctrl_off, np.int32),
                                              device=device)}
        for k in self.FIELDS:
            a = np.ascontiguousarray(getattr(ps, k), np.float64)
            if a.size == 0:
                a = np.zeros(1)
            self.t[k] = torch.as_tensor(a, device=device).contiguous()
        self.struct = LbmParticles(ps.n, *[_ptr(self.t[k]) for k in ("ctrl_off",) + self.FIELDS])

    def set_state(self, ps):
        torch = _torch()
        for k in ("pos", "quat", "vel", "omega", "world_pts"):
            a = np.ascontiguousarray(getattr(ps, k), np.float64)
            if a.size:
                self.t[k].copy_(torch.as_tensor(a).reshape(self.t[k].shape))

    def to_host(self, ps):
        out = ps.copy()
        for k in ("pos", "quat", "vel", "omega", "world_pts"):
            if getattr(ps, k).size:
                setattr(out, k, self.t[k].cpu().numpy().reshape(getattr(ps, k).shape).copy())
        return out


class DeviceTrajectory:
    """A sequence of particle states of one particle set, resident on the
    device: the shape data once, pose and world control points per state
    ([T, ...] tensors), velocities either per state or one array for all.
    Item t is an object with the lbm_particles `struct` of state t, usable
    wherever a DeviceParticles is."""

    class _State:
        def __init__(self, struct, owner):
            self.struct = struct
            self._owner = owner   # keeps the tensors alive

    def __init__(self, states, vel=None, omega=None, device="cuda"):
        torch = _torch()
        self.base = DeviceParticles(states[0], device=device)
        self.n = states[0].n
        stack = lambda k: torch.as_tensor(
            np.ascontiguousarray(np.stack([getattr(s, k) for s in states]), np.float64),
            device=device)
        self.pos, self.quat, self.world = stack("pos"), stack("quat"), stack("world_pts")
        one = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float64), device=device)
        self.vel = one(states[0].vel if vel is None else vel)
        self.omega = one(states[0].omega if omega is None else omega)
        b = self.base.t
        self._items = []
        for t in range(len(states)):
            st = LbmParticles(self.n, _ptr(b["ctrl_off"]), _ptr(b["body_pts"]), _ptr(b["K"]),
                              _ptr(b["c0"]), _ptr(b["rs"]), _ptr(b["mass"]), _ptr(b["volume"]),
                              _ptr(b["inertia"]), _ptr(self.pos[t]), _ptr(self.quat[t]),
                              _ptr(self.vel), _ptr(self.omega), _ptr(self.world[t]))
            self._items.append(self._State(st, self))

    def __len__(self):
        return len(self._items)

    def __getitem__(self, t):
        return self._items[t]


class Lattice:
    """A lattice, its caller-owned device buffers and a library context."""

    def __init__(self, lat, n_particles=0, n_ctrl=0, box_half=2, storage="f32",
                 treatments=TREAT_VIBB | TREAT_MISSING, h16_scale=0.0, device="cuda",
                 classify="auto", lattice=19, exact_forces=False):
        """lattice: 19 (D3Q19) or 15 (D3Q15, the paper's Sec. 2.2); exact_forces:
        sum the link pass's momentum exchange exactly in 128-bit integers, so
        that forces and torques are the same bits on every run."""
        torch = _torch()
        self.torch = torch
        self.device = torch.device(device)
        self.storage = storage
        cfg = LbmConfig()
        cfg.nx, cfg.ny, cfg.nz = lat.nx, lat.ny, lat.nz
        cfg.periodic = (ctypes.c_int32 * 3)(*[int(bool(v)) for v in lat.periodic])
        cfg.tau = float(lat.tau)
        cfg.rho0 = float(lat.rho0)
        cfg.u0 = (ctypes.c_double * 3)(*map(float, lat.u0))
        cfg.body_force = (ctypes.c_double * 3)(*map(float, lat.body_force))
        cfg.storage = STORAGE[storage]
        cfg.treatments = int(treatments)
        cfg.n_particles = int(n_particles)
        cfg.n_ctrl = int(n_ctrl)
        cfg.box_half = int(box_half)
        cfg.h16_scale = float(h16_scale)
        cfg.classify_mode = CLASSIFY[classify]
        cfg.lattice = int(lattice)
        cfg.force_sum = FORCE_SUM_EXACT if exact_forces else FORCE_SUM_ATOMIC
        self.Q = 15 if int(lattice) == 15 else 19
        with torch.cuda.device(self.device):
            cfg.stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        self.cfg = cfg
        self.sizes = lbm_query_sizes(cfg)
        self.ncell = int(self.sizes.ncell)
        u8 = dict(dtype=torch.uint8, device=self.device)
        self.f = [torch.empty(self.sizes.population_bytes, **u8) for _ in range(2)]
        self.own = [torch.empty(self.sizes.owner_bytes // 4, dtype=torch.int32, device=self.device)
                    for _ in range(2)]
        self.flag = torch.empty(self.sizes.flag_bytes, **u8)
        self.mom = torch.empty(self.sizes.moment_bytes, **u8)
        bufs = LbmBuffers((_P * 2)(*[t.data_ptr() for t in self.f]),
                          (_P * 2)(*[t.data_ptr() for t in self.own]), self.flag.data_ptr(),
                          self.mom.data_ptr())
        self.ctx = lbm_init(cfg, bufs)
        self.n_particles = int(n_particles)
        self.F = torch.zeros((max(n_particles, 1), 3), dtype=torch.float64, device=self.device)
        self.T = torch.zeros_like(self.F)

    @classmethod
    def for_particles(cls, lat, ps, **kw):
        return cls(lat, n_particles=ps.n, n_ctrl=len(ps.K), box_half=ps.box_half(), **kw)

    # the five calls of the hot path
    def classify(self, parts: DeviceParticles, sync: bool = True) -> LbmCounts | None:
        """With sync=False, lbm_classify_nodes_async: no counts, and errors
        are raised by the next synchronising call."""
        if not sync:
            lbm_classify_nodes_async(self.ctx, parts.struct)
            return None
        return lbm_classify_nodes(self.ctx, parts.struct)

    def step(self, parts: DeviceParticles):
        lbm_step(self.ctx, parts.struct)

    def forces(self, F=None, T=None):
        """The last step's F^h, T^h (device, [n][3] float64 each), copied into
        F and T when given (contiguous device tensors), else into the
        lattice's own buffers."""
        if F is None:
            F, T = self.F, self.T
        lbm_particle_forces(self.ctx, F, T)
        return F[: self.n_particles], T[: self.n_particles]

    def dem(self, parts: DeviceParticles, n_sub: int, dt: float, prm: DemParams):
        dem_step(self.ctx, parts.struct, n_sub, dt, prm)

    def step_dem(self, parts: DeviceParticles, n_sub: int, dt: float, prm: DemParams):
        """lbm_step_dem: the step, with the DEM sub-cycle beside its
        stream-collide pass."""
        lbm_step_dem(self.ctx, parts.struct, n_sub, dt, prm)

    def dem_noalloc(self, parts: DeviceParticles, n_sub: int, dt: float, prm: DemParams):
        """dem_step_noalloc: the same substeps with the static work space."""
        dem_step_noalloc(self.ctx, parts.struct, n_sub, dt, prm)

    def sync(self):
        lbm_synchronize(self.ctx)

    def profile(self, on: bool):
        _check(load().lbm_profile_enable(self.ctx, int(bool(on))), self.ctx)

    def profile_read(self) -> dict:
        out = LbmProfile()
        _check(load().lbm_profile_read(self.ctx, ctypes.byref(out)), self.ctx)
        return {name: (out.ms[i], int(out.launches[i])) for i, name in enumerate(PHASES)}

    # inspection
    def owner(self) -> np.ndarray:
        out = self.torch.empty(self.ncell, dtype=self.torch.int32, device=self.device)
        _check(load().lbm_get_owner(self.ctx, _ptr(out)), self.ctx)
        return out.cpu().numpy()

    def populations(self, nodes=None) -> np.ndarray:
        """FP64 populations [Q][ncell]; with nodes (indices), only those
        columns are copied to the host."""
        out = self.torch.empty((self.Q, self.ncell), dtype=self.torch.float64, device=self.device)
        _check(load().lbm_get_populations(self.ctx, _ptr(out)), self.ctx)
        if nodes is not None:
            idx = self.torch.as_tensor(np.asarray(nodes, np.int64), device=self.device)
            out = out[:, idx]
        return out.cpu().numpy()

    def moments(self):
        """(rho [ncell], u [ncell][3]) in FP64 from the last collision."""
        rho = self.torch.empty(self.ncell, dtype=self.torch.float64, device=self.device)
        u = self.torch.empty((self.ncell, 3), dtype=self.torch.float64, device=self.device)
        _check(load().lbm_get_moments(self.ctx, _ptr(rho), _ptr(u)), self.ctx)
        return rho.cpu().numpy(), u.cpu().numpy()

    def set_populations(self, f: np.ndarray):
        t = self.torch.as_tensor(np.ascontiguousarray(f, np.float64), device=self.device)
        _check(load().lbm_set_populations(self.ctx, _ptr(t)), self.ctx)
        self.sync()

    def links(self):
        """Link records sorted into canonical order (particle, node, d)."""
        n = ctypes.c_int64()
        rc = load().lbm_get_links(self.ctx, 0, None, None, None, None, None, ctypes.byref(n))
        if rc not in (LBM_OK, LBM_ECAPACITY):
            _check(rc, self.ctx)
        m = int(n.value)
        torch = self.torch
        if m == 0:
            z = np.zeros(0)
            return dict(node=z.astype(np.int32), d=z.astype(np.int8), kind=z.astype(np.int8),
                        part=z.astype(np.int32), q=z)
        node = torch.empty(m, dtype=torch.int32, device=self.device)
        d = torch.empty(m, dtype=torch.int8, device=self.device)
        kind = torch.empty(m, dtype=torch.int8, device=self.device)
        part = torch.empty(m, dtype=torch.int32, device=self.device)
        q = torch.empty(m, dtype=torch.float64, device=self.device)
        _check(load().lbm_get_links(self.ctx, m, _ptr(node), _ptr(d), _ptr(kind), _ptr(part),
                                    _ptr(q), ctypes.byref(n)), self.ctx)
        out = dict(node=node.cpu().numpy(), d=d.cpu().numpy(), kind=kind.cpu().numpy(),
                   part=part.cpu().numpy(), q=q.cpu().numpy())
        order = np.lexsort((out["d"], out["node"], out["part"]))
        return {k: v[order] for k, v in out.items()}

    def refill(self):
        n = ctypes.c_int64()
        rc = load().lbm_get_refill(self.ctx, 0, None, None, ctypes.byref(n))
        if rc not in (LBM_OK, LBM_ECAPACITY):
            _check(rc, self.ctx)
        m = int(n.value)
        if m == 0:
            return np.zeros(0, np.int32), np.zeros(0, np.int32)
        torch = self.torch
        node = torch.empty(m, dtype=torch.int32, device=self.device)
        part = torch.empty(m, dtype=torch.int32, device=self.device)
        _check(load().lbm_get_refill(self.ctx, m, _ptr(node), _ptr(part), ctypes.byref(n)),
               self.ctx)
        node, part = node.cpu().numpy(), part.cpu().numpy()
        o = np.argsort(node, kind="stable")
        return node[o], part[o]

    # differentiation form
    def checkpoint(self):
        t = self.torch.empty(self.sizes.checkpoint_bytes, dtype=self.torch.uint8, device=self.device)
        _check(load().lbm_checkpoint_save(self.ctx, _ptr(t)), self.ctx)
        return t

    def restore(self, t):
        _check(load().lbm_checkpoint_load(self.ctx, _ptr(t)), self.ctx)

    def dem_checkpoint(self):
        t = self.torch.empty(max(self.sizes.dem_checkpoint_bytes, 1), dtype=self.torch.uint8,
                             device=self.device)
        _check(load().lbm_dem_checkpoint_save(self.ctx, _ptr(t)), self.ctx)
        return t

    def dem_restore(self, t):
        _check(load().lbm_dem_checkpoint_load(self.ctx, _ptr(t)), self.ctx)

    def geometry_bytes(self):
        """(bytes, tag) of a geometry snapshot for the current list capacities."""
        n, tag = ctypes.c_size_t(), ctypes.c_uint64()
        _check(load().lbm_geometry_bytes(self.ctx, ctypes.byref(n), ctypes.byref(tag)), self.ctx)
        return int(n.value), int(tag.value)

    def geometry_save(self, t=None):
        """The last classification's geometry into t (a new device buffer if
        None); returns (t, tag)."""
        n, tag = self.geometry_bytes()
        if t is None:
            t = self.torch.empty(n, dtype=self.torch.uint8, device=self.device)
        _check(load().lbm_geometry_save(self.ctx, _ptr(t)), self.ctx)
        return t, tag

    def geometry_load(self, snap, parts: "DeviceParticles"):
        """Stand in for classify(parts) with a snapshot (t, tag) taken at that pose."""
        t, tag = snap
        _check(load().lbm_geometry_load(self.ctx, _ptr(t), ctypes.c_uint64(tag),
                                        ctypes.byref(parts.struct)), self.ctx)

    def tape_begin(self, steps: int):
        _check(load().lbm_tape_begin(self.ctx, int(steps)), self.ctx)

    def adjoint_field(self):
        """A zero adjoint field (Q planes in the storage's arithmetic)."""
        dt = self.torch.float64 if self.storage == "f64" else self.torch.float32
        es = 8 if self.storage == "f64" else 4
        return self.torch.zeros(self.sizes.adjoint_bytes // es, dtype=dt, device=self.device)

    def adjoint(self, parts: "DeviceParticles", weights: np.ndarray, lam, grad, gpos=None):
        """gpos: None, or a zeroed device FP64 tensor [(T + 1), n, 6] that
        receives (dJ/dx_p, dJ/dtheta_p) of each taped step's pose (and of
        parts)."""
        w = np.ascontiguousarray(weights, np.float64).reshape(-1)
        _check(load().lbm_adjoint(self.ctx, ctypes.byref(parts.struct),
                                  w.ctypes.data_as(ctypes.c_void_p), _ptr(lam), _ptr(grad),
                                  None if gpos is None else _ptr(gpos)),
               self.ctx)

    def adjoint_coupled(self, parts: "DeviceParticles", weights: np.ndarray, prm: DemParams,
                        n_sub: int, dt: float, lam, grad, sigma, sigma_contact=None):
        """Adjoint of a free-moving run over the taped steps (each followed by
        dem with these arguments); sigma: device FP64 [n, 12], in/out;
        sigma_contact: device FP64 [n, contact_adjoint_bytes / 8], in/out, or
        None for zero."""
        w = np.ascontiguousarray(weights, np.float64).reshape(-1)
        _check(load().lbm_adjoint_coupled(self.ctx, ctypes.byref(parts.struct),
                                          w.ctypes.data_as(ctypes.c_void_p), ctypes.byref(prm),
                                          int(n_sub), float(dt), _ptr(lam), _ptr(grad),
                                          _ptr(sigma),
                                          None if sigma_contact is None else _ptr(sigma_contact)),
               self.ctx)

    def contact_adjoint(self):
        """A zero contact-state adjoint for adjoint_coupled."""
        n = max(self.sizes.contact_adjoint_bytes // 8, 1)
        return self.torch.zeros(n, dtype=self.torch.float64, device=self.device)

    def close(self):
        if getattr(self, "ctx", None):
            lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
