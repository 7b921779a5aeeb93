"""ctypes front end of the FP64 CPU oracle (mdlbm_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the CPU
baseline timing of the benchmark, never by the product path.  It does not
import the HIP package; it takes plain numpy arrays (any object with the
attributes of a particle set works).

The coupled loop it drives, one lattice step n -> n+1:

    step(P^n)        unknowns on links L^n, force/torque, stream + collide
    (DEM or a prescribed trajectory gives P^{n+1})
    classify(P^{n+1}) owners, links L^{n+1}, refill of nodes uncovered since n

which is the order of Sec. 2.3 (boundary condition, momentum exchange,
sub-cycled DEM, refilling) written as one loop.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from pathlib import Path

import numpy as np

HERE = Path(__file__).resolve().parent
SRC = HERE / "mdlbm_oracle.c"
BUILD = HERE / "_build"
LIB = BUILD / "libmdlbm_oracle.so"

KIND_VIBB, KIND_HALFWAY, KIND_MISSING = 0, 1, 2
TREAT_VIBB, TREAT_MISSING, TREAT_EXACT_Q, TREAT_NEQ_SPLIT = 1, 2, 4, 8

_lib = None


def build(force: bool = False) -> Path:
    """Compile the oracle with gcc (IEEE double, no FMA contraction, OpenMP)."""
    BUILD.mkdir(exist_ok=True)
    if force or not LIB.exists() or LIB.stat().st_mtime < SRC.stat().st_mtime:
        tmp = LIB.with_suffix(f".so.tmp{os.getpid()}")
        subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                        "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wno-unknown-pragmas",
                        "-o", str(tmp), str(SRC), "-lm"], check=True)
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(str(LIB))
        P = ctypes.c_void_p
        L.ora_metaball.restype = ctypes.c_double
        L.ora_metaball.argtypes = [ctypes.c_int, P, P, P]
        L.ora_vibb.restype = ctypes.c_double
        L.ora_vibb.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                               ctypes.c_double, P, ctypes.c_double, ctypes.c_double, P, P,
                               ctypes.c_int]
        L.ora_links.restype = ctypes.c_long
        L.ora_links.argtypes = [P, P, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P, P, P, P, P,
                                ctypes.c_long, P, P, P, P, P]
        L.ora_step.restype = ctypes.c_int
        L.ora_step.argtypes = [P, P, ctypes.c_int, ctypes.c_int, ctypes.c_double, P, ctypes.c_double, P, P,
                               ctypes.c_long, P, P, P, P, P, ctypes.c_int, P, P, P, P, P, P, P]
        L.ora_refill.restype = ctypes.c_long
        L.ora_refill.argtypes = [P, P, ctypes.c_int, ctypes.c_double, P, ctypes.c_double, P, P, P,
                                 ctypes.c_int, P, P, P, P, ctypes.c_long, P]
        L.ora_classify.restype = None
        L.ora_classify.argtypes = [P, P, ctypes.c_int, P, P, P, P, P, P]
        L.ora_moments.restype = None
        L.ora_moments.argtypes = [P, ctypes.c_int, P, P, P, P]
        L.ora_init_equilibrium.restype = None
        L.ora_init_equilibrium.argtypes = [P, ctypes.c_int, ctypes.c_double, P, P]
        L.ora_stencil.restype = ctypes.c_int
        L.ora_stencil.argtypes = [ctypes.c_int, P, P, P]
        L.ora_dem_step.restype = None
        L.ora_dem_step.argtypes = [ctypes.c_int] + [P] * 19 + [P, P, ctypes.c_int, ctypes.c_double]
        L.ora_num_threads.restype = ctypes.c_int
        L.ora_set_num_threads.restype = None
        L.ora_set_num_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"], "arrays passed to the oracle must be contiguous"
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def stencil(Q: int = 19):
    e = np.zeros((Q, 3), np.int32)
    w = np.zeros(Q, np.float64)
    opp = np.zeros(Q, np.int32)
    lib().ora_stencil(Q, _p(e), _p(w), _p(opp))
    return e, w, opp


def metaball(pts, K, X) -> float:
    pts = _c(pts, np.float64)
    K = _c(K, np.float64)
    X = _c(X, np.float64)
    return lib().ora_metaball(len(K), _p(pts), _p(K), _p(X))


def vibb(d, q, fd_f, rho_f, u_f, fd_ff, rho_ff, u_ff, uw, Q=19, treat=0) -> float:
    return lib().ora_vibb(Q, d, q, fd_f, rho_f, _p(_c(u_f, np.float64)), fd_ff, rho_ff,
                          _p(_c(u_ff, np.float64)), _p(_c(uw, np.float64)), int(treat))


def num_threads() -> int:
    return lib().ora_num_threads()


def set_num_threads(n: int) -> None:
    """Threads of the oracle's parallel loops (their results do not depend
    on it: force sums are serial in link order)."""
    lib().ora_set_num_threads(int(n))


class Links:
    """Link records in canonical order (particle, solid node x_s, direction d)."""

    def __init__(self, node, d, kind, part, q):
        self.node, self.d, self.kind, self.part, self.q = node, d, kind, part, q

    def __len__(self):
        return len(self.node)


class DemParams:
    def __init__(self, kn=0.0, eta_n=0.0, kt=0.0, eta_t=0.0, mu_s=0.3, ctol=1e-3,
                 newton_tol=1e-12, newton_iter=50, gravity=(0.0, 0.0, 0.0), rho_f=1.0):
        self.kn, self.eta_n, self.kt, self.eta_t, self.mu_s = kn, eta_n, kt, eta_t, mu_s
        self.ctol, self.newton_tol, self.newton_iter = ctol, newton_tol, newton_iter
        self.gravity, self.rho_f = tuple(gravity), rho_f

    def packed(self) -> np.ndarray:
        return np.array([self.kn, self.eta_n, self.kt, self.eta_t, self.mu_s, self.ctol,
                         self.newton_tol, float(self.newton_iter), *self.gravity, self.rho_f],
                        np.float64)


class Oracle:
    """FP64 lattice + particles.  `f` is Q x N post-collision populations
    (x fastest), `owner` is 0 for fluid and p+1 for a node of particle p."""

    def __init__(self, lat, Q: int = 19, treat: int = TREAT_VIBB | TREAT_MISSING,
                 fields: bool = True):
        """fields=False keeps the geometry only (owners, links, and the refill
        set by its definition: solid before, fluid now), without population
        arrays, for lattices whose FP64 populations would not fit in memory."""
        self.dims = np.array([lat.nx, lat.ny, lat.nz], np.int32)
        self.per = np.array([int(bool(v)) for v in lat.periodic], np.int32)
        self.N = int(lat.nx) * int(lat.ny) * int(lat.nz)
        self.Q = Q
        self.treat = treat
        self.tau = float(lat.tau)
        self.rho0 = float(lat.rho0)
        self.Fb = _c(lat.body_force, np.float64)
        self.f = self.fprev = None
        if fields:
            self.f = np.zeros((Q, self.N), np.float64)
            lib().ora_init_equilibrium(_p(self.dims), Q, self.rho0, _p(_c(lat.u0, np.float64)),
                                       _p(self.f))
            self.fprev = self.f.copy()
        self.owner = np.zeros(self.N, np.int32)
        self.owner_prev = None
        self.links = Links(*(np.zeros(0, t) for t in (np.int32, np.int8, np.int8, np.int32,
                                                      np.float64)))
        self.refill_nodes = np.zeros(0, np.int32)
        self.unknown = np.zeros(0)
        self.F = np.zeros((0, 3))
        self.T = np.zeros((0, 3))

    # -- geometry ----------------------------------------------------------
    def _particle_arrays(self, ps):
        return (_c(ps.ctrl_off, np.int32), _c(ps.world_pts, np.float64), _c(ps.K, np.float64),
                _c(ps.c0, np.float64), _c(ps.pos, np.float64))

    def owners(self, ps) -> np.ndarray:
        off, pts, K, c0, xp = self._particle_arrays(ps)
        own = np.zeros(self.N, np.int32)
        lib().ora_classify(_p(self.dims), _p(self.per), len(c0), _p(off), _p(pts), _p(K), _p(c0),
                           _p(xp), _p(own))
        return own

    def build_links(self, ps, owner) -> Links:
        off, pts, K, c0, xp = self._particle_arrays(ps)
        cap = 1 << 16
        while True:
            arrs = [np.zeros(cap, t) for t in (np.int32, np.int8, np.int8, np.int32, np.float64)]
            n = lib().ora_links(_p(self.dims), _p(self.per), self.Q, self.treat, len(c0), _p(off),
                                _p(pts), _p(K), _p(c0), _p(xp), _p(owner), cap,
                                *[_p(a) for a in arrs])
            if n <= cap:
                return Links(*[a[:n].copy() for a in arrs])
            cap = int(n) + 16

    def classify(self, ps, refill: bool = True):
        """Owners and links for particle state ps; refill nodes uncovered since
        the previous classification (not on the first call)."""
        own = self.owners(ps)
        first = self.owner_prev is None and not getattr(self, "_classified", False)
        if refill and not first and self.f is None:
            self.refill_nodes = np.flatnonzero((self.owner > 0) & (own == 0)).astype(np.int32)
        elif refill and not first:
            cap = max(1, self.N)
            nodes = np.zeros(cap, np.int32)
            n = lib().ora_refill(_p(self.dims), _p(self.per), self.Q, self.tau, _p(self.Fb),
                                 self.rho0, _p(self.fprev), _p(self.owner), _p(own), ps.n,
                                 _p(_c(ps.pos, np.float64)), _p(_c(ps.vel, np.float64)),
                                 _p(_c(ps.omega, np.float64)), _p(self.f), cap, _p(nodes))
            self.refill_nodes = nodes[:n].copy()
        else:
            self.refill_nodes = np.zeros(0, np.int32)
        self._classified = True
        self.owner_prev = self.owner
        self.owner = own
        self.links = self.build_links(ps, own)
        return self

    # -- lattice step ------------------------------------------------------
    def step(self, ps):
        L = self.links
        nl = len(L)
        fout = np.empty_like(self.f)
        unk = np.zeros(max(nl, 1))
        F = np.zeros((ps.n, 3))
        T = np.zeros((ps.n, 3))
        rc = lib().ora_step(_p(self.dims), _p(self.per), self.Q, self.treat, self.tau, _p(self.Fb),
                            self.rho0,
                            _p(self.f), _p(self.owner), nl, _p(L.node), _p(L.d), _p(L.kind),
                            _p(L.part), _p(L.q), ps.n, _p(_c(ps.pos, np.float64)),
                            _p(_c(ps.vel, np.float64)), _p(_c(ps.omega, np.float64)), _p(fout),
                            _p(unk), _p(F), _p(T))
        if rc != 0:
            raise RuntimeError("oracle step: a solid source node has no link")
        self.fprev = self.f
        self.f = fout
        self.unknown = unk[:nl]
        self.F, self.T = F, T
        return F, T

    def moments(self):
        rho = np.zeros(self.N)
        u = np.zeros((self.N, 3))
        lib().ora_moments(_p(self.dims), self.Q, _p(self.Fb), _p(self.f), _p(rho), _p(u))
        return rho, u

    def field(self, arr):
        """View an N-vector as (nz, ny, nx)."""
        return arr.reshape(int(self.dims[2]), int(self.dims[1]), int(self.dims[0]))


class OracleDEM:
    """FP64 DEM state for a particle set (contact histories held here)."""

    def __init__(self, ps, lat):
        self.np = ps.n
        self.dims = np.array([lat.nx, lat.ny, lat.nz], np.int32)
        self.per = np.array([int(bool(v)) for v in lat.periodic], np.int32)
        self.hpp = np.zeros((max(self.np, 1) ** 2) * 8)
        self.hpw = np.zeros(max(self.np, 1) * 6 * 8)
        self.fc = np.zeros((self.np, 3))
        self.tc = np.zeros((self.np, 3))

    def step(self, ps, Fh, Th, prm: DemParams, n_sub: int, dt: float):
        arrs = {k: _c(getattr(ps, k), np.float64) for k in
                ("body_pts", "K", "rs", "mass", "volume", "inertia", "pos", "quat", "vel",
                 "omega", "world_pts")}
        off = _c(ps.ctrl_off, np.int32)
        Fh = _c(Fh, np.float64)
        Th = _c(Th, np.float64)
        lib().ora_dem_step(self.np, _p(off), _p(arrs["body_pts"]), _p(arrs["K"]), _p(arrs["rs"]),
                           _p(arrs["mass"]), _p(arrs["volume"]), _p(arrs["inertia"]),
                           _p(arrs["pos"]), _p(arrs["quat"]), _p(arrs["vel"]), _p(arrs["omega"]),
                           _p(arrs["world_pts"]), _p(self.fc), _p(self.tc), _p(Fh), _p(Th),
                           _p(self.hpp), _p(self.hpw), _p(prm.packed()), _p(self.dims),
                           _p(self.per), int(n_sub), float(dt))
        for k in ("pos", "quat", "vel", "omega", "world_pts"):
            setattr(ps, k, arrs[k])
        return ps
