"""Seeded synthetic inputs shared by the GPU path, its tests and the CPU oracle.

This module only *prepares inputs*: lattice sizes, particle shapes (metaball
control points x_i and weights K_i, Sec. 2.1.2), rigid-body properties and
placements, and prescribed trajectories for replay runs.  It contains none of
the lattice update, boundary reconstruction, force evaluation, refilling or
DEM contact arithmetic; both the HIP library and the oracle receive the arrays
built here and nothing else from it.

Rigid-body inputs (volume, mass, principal inertia, the surface level c0) are
properties of a shape that the paper treats as given (Sec. 3.2 quotes the
particle's volume and density).  They are obtained here once per shape by a
sub-voxel point-count quadrature of the body {x : sum_i K_i/|x-x_i|^2 >= c0}.

Conventions (lattice units, dx = dt = 1):
  * node (i, j, k) sits at coordinates (i, j, k); x is the fastest index;
  * a non-periodic axis has walls half a cell outside the first and last node
    (at -0.5 and n-0.5);
  * quaternions are (w, x, y, z) and rotate body-frame vectors into the world;
  * angular velocities are world-frame vectors.
"""
from __future__ import annotations

import dataclasses
import hashlib
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "LatticeSpec", "ParticleSet", "quat_to_matrix", "random_quaternion",
    "sphere_shape", "metaball_shape", "make_particles", "prescribed_state",
    "config_c1", "config_c2", "config_c3", "config_c4", "config_c5",
    "square_metaball", "config_dkt", "config_floor_pair",
    "tiny_case", "WORKLOADS", "drag_case", "DRAG_CASES", "fingerprint",
]


@dataclass
class LatticeSpec:
    nx: int
    ny: int
    nz: int
    periodic: tuple = (0, 0, 0)
    tau: float = 0.8
    rho0: float = 1.0
    u0: tuple = (0.0, 0.0, 0.0)
    body_force: tuple = (0.0, 0.0, 0.0)

    @property
    def ncell(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def dims(self):
        return (self.nx, self.ny, self.nz)


@dataclass
class Shape:
    """Body-frame metaball: control points (principal frame, origin at the
    centroid), weights, surface level c0, sphero radius R_s and rigid-body
    properties for unit density."""
    pts: np.ndarray
    K: np.ndarray
    c0: float
    rs: float
    volume: float
    inertia_unit: np.ndarray  # principal moments per unit density
    radius: float             # max distance from the origin of {M >= c0}


@dataclass
class ParticleSet:
    ctrl_off: np.ndarray   # int32 (n+1,)
    body_pts: np.ndarray   # f64 (m,3)
    K: np.ndarray          # f64 (m,)
    c0: np.ndarray         # f64 (n,)
    rs: np.ndarray         # f64 (n,)
    volume: np.ndarray     # f64 (n,)
    mass: np.ndarray       # f64 (n,)
    inertia: np.ndarray    # f64 (n,3)
    pos: np.ndarray        # f64 (n,3)
    quat: np.ndarray       # f64 (n,4)
    vel: np.ndarray        # f64 (n,3)
    omega: np.ndarray      # f64 (n,3)
    radius: np.ndarray     # f64 (n,) bound on |x - x_p| over the body
    world_pts: np.ndarray = field(default=None)  # f64 (m,3)

    @property
    def n(self) -> int:
        return len(self.c0)

    def copy(self) -> "ParticleSet":
        return dataclasses.replace(
            self, **{f.name: (None if getattr(self, f.name) is None
                              else np.array(getattr(self, f.name), copy=True))
                     for f in dataclasses.fields(self)})

    def refresh_world(self) -> None:
        self.world_pts = world_points(self.pos, self.quat, self.body_pts, self.ctrl_off)

    def box_half(self) -> int:
        """Half-width h of the per-particle node box [floor(x_p)-h, floor(x_p)+h]:
        every body point lies within `radius` < h - 1 of x_p."""
        if self.n == 0:
            return 2
        return int(np.floor(self.radius.max())) + 3


# ----------------------------------------------------------------------------
# rigid transforms
# ----------------------------------------------------------------------------

def quat_to_matrix(q: np.ndarray) -> np.ndarray:
    q = np.asarray(q, dtype=np.float64)
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    R = np.empty(q.shape[:-1] + (3, 3))
    R[..., 0, 0] = 1 - 2 * (y * y + z * z)
    R[..., 0, 1] = 2 * (x * y - w * z)
    R[..., 0, 2] = 2 * (x * z + w * y)
    R[..., 1, 0] = 2 * (x * y + w * z)
    R[..., 1, 1] = 1 - 2 * (x * x + z * z)
    R[..., 1, 2] = 2 * (y * z - w * x)
    R[..., 2, 0] = 2 * (x * z - w * y)
    R[..., 2, 1] = 2 * (y * z + w * x)
    R[..., 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def quat_mul(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    aw, ax, ay, az = a
    bw, bx, by, bz = b
    return np.array([aw * bw - ax * bx - ay * by - az * bz,
                     aw * bx + ax * bw + ay * bz - az * by,
                     aw * by - ax * bz + ay * bw + az * bx,
                     aw * bz + ax * by - ay * bx + az * bw])


def random_quaternion(rng: np.random.Generator) -> np.ndarray:
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    if q[0] < 0:
        q = -q
    return q


def world_points(pos, quat, body_pts, ctrl_off) -> np.ndarray:
    out = np.empty_like(body_pts)
    R = quat_to_matrix(quat)
    for p in range(len(pos)):
        a, b = ctrl_off[p], ctrl_off[p + 1]
        out[a:b] = pos[p] + body_pts[a:b] @ R[p].T
    return out


# ----------------------------------------------------------------------------
# shapes
# ----------------------------------------------------------------------------

def _field(pts: np.ndarray, K: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Implicit shape function at sample points X (..., 3); shape prep only."""
    acc = np.zeros(X.shape[:-1])
    for p, k in zip(pts, K):
        r2 = ((X - p) ** 2).sum(-1)
        with np.errstate(divide="ignore"):
            acc += k / r2
    return acc


def _mass_properties(pts, K, c0, samples_per_unit: float, reach: float):
    """Point-count quadrature of the body {field >= c0}: volume, centroid and
    inertia tensor per unit density."""
    lo = pts.min(0) - reach
    hi = pts.max(0) + reach
    h = 1.0 / samples_per_unit
    axes = [np.arange(lo[a] + 0.5 * h, hi[a], h) for a in range(3)]
    vol = 0.0
    s1 = np.zeros(3)
    s2 = np.zeros((3, 3))
    rmax2 = 0.0
    # slab by slab in z to bound memory
    X, Y = np.meshgrid(axes[0], axes[1], indexing="ij")
    for z in axes[2]:
        P = np.stack([X, Y, np.full_like(X, z)], -1)
        inside = _field(pts, K, P) >= c0
        if not inside.any():
            continue
        Q = P[inside]
        vol += len(Q)
        s1 += Q.sum(0)
        s2 += Q.T @ Q
        rmax2 = max(rmax2, float(((Q - pts.mean(0)) ** 2).sum(-1).max()))
    dv = h ** 3
    V = vol * dv
    c = s1 / vol
    second = s2 * dv - V * np.outer(c, c)
    inertia = np.trace(second) * np.eye(3) - second
    return V, c, inertia


def body_radius(pts: np.ndarray, K: np.ndarray, c0: float) -> float:
    """Radius about the origin beyond which no point reaches level c0.

    At distance d > |x_i| from the origin, |x - x_i| >= d - |x_i|, so
    M(x) <= sum_i K_i / (d - |x_i|)^2, which decreases in d; the root of that
    bound at c0 (bisection) bounds the body."""
    b = np.sqrt((np.asarray(pts, float) ** 2).sum(-1))
    K = np.asarray(K, float)

    def bound(d):
        return float((K / (d - b) ** 2).sum())

    lo = b.max() + 1e-9
    hi = b.max() + np.sqrt(K.sum() / c0) + 1.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if bound(mid) >= c0:
            lo = mid
        else:
            hi = mid
    return hi


def _finish_shape(pts, K, c0, rs, samples_per_unit) -> Shape:
    reach = float(np.sqrt(K.sum() / c0)) + 1.0
    V, c, I = _mass_properties(pts, K, c0, samples_per_unit, reach)
    evals, evecs = np.linalg.eigh(I)
    if np.linalg.det(evecs) < 0:
        evecs[:, 0] = -evecs[:, 0]
    body = (pts - c) @ evecs            # principal frame, centroid origin
    radius = body_radius(body, K, c0)
    return Shape(pts=body, K=K.copy(), c0=float(c0), rs=float(rs), volume=V,
                 inertia_unit=evals, radius=radius)


def sphere_shape(diameter: float, rs: float) -> Shape:
    """One control point: internal radius r - R_s, surface level c0 such that
    {M >= c0} is the ball of the given diameter (K_0 = (d/2 - R_s)^2, Sec. 3.1)."""
    r = 0.5 * diameter
    K = np.array([(r - rs) ** 2])
    c0 = ((r - rs) / r) ** 2
    V = 4.0 / 3.0 * np.pi * r ** 3
    Iu = 0.4 * V * r * r
    return Shape(pts=np.zeros((1, 3)), K=K, c0=float(c0), rs=float(rs), volume=V,
                 inertia_unit=np.full(3, Iu), radius=r)


def metaball_shape(pts: np.ndarray, K: np.ndarray, rs: float, *, d_eq: float | None = None,
                   length: float | None = None, axis: np.ndarray | None = None,
                   samples_per_unit: float = 2.0) -> Shape:
    """Scale a unit metaball (x_i -> s x_i, K_i -> s^2 K_i leaves its level sets
    similar) so that either its volume-equivalent diameter or its extent along
    ``axis`` matches, then set c0 so that the level set {M >= c0} is the
    internal body {M >= 1} grown by roughly R_s."""
    pts = np.asarray(pts, float)
    K = np.asarray(K, float)
    # unit-scale internal body
    reach = float(np.sqrt(K.sum())) + 1.0
    if d_eq is not None:
        V1, _, _ = _mass_properties(pts, K, 1.0, 24.0, reach)
        s = ((np.pi / 6.0) * (d_eq - 2 * rs) ** 3 / V1) ** (1.0 / 3.0)
    else:
        ax = np.asarray(axis, float) / np.linalg.norm(axis)
        t = np.linspace(-4 * reach, 4 * reach, 20001)
        X = pts.mean(0) + t[:, None] * ax
        inside = _field(pts, K, X) >= 1.0
        ext = t[inside].max() - t[inside].min()
        s = (length - 2 * rs) / ext
    pts_s = pts * s
    K_s = K * s * s
    V_int, _, _ = _mass_properties(pts_s, K_s, 1.0, samples_per_unit,
                                   float(np.sqrt(K_s.sum())) + 1.0)
    r_int = (3.0 * V_int / (4.0 * np.pi)) ** (1.0 / 3.0)
    c0 = (r_int / (r_int + rs)) ** 2
    return _finish_shape(pts_s, K_s, c0, rs, samples_per_unit)


def make_particles(shapes, pos, quat, rho_p, vel=None, omega=None) -> ParticleSet:
    n = len(shapes)
    pos = np.asarray(pos, float).reshape(n, 3)
    quat = np.asarray(quat, float).reshape(n, 4)
    rho_p = np.broadcast_to(np.asarray(rho_p, float), (n,))
    counts = [len(s.K) for s in shapes]
    off = np.zeros(n + 1, np.int32)
    off[1:] = np.cumsum(counts)
    ps = ParticleSet(
        ctrl_off=off,
        body_pts=np.concatenate([s.pts for s in shapes]) if n else np.zeros((0, 3)),
        K=np.concatenate([s.K for s in shapes]) if n else np.zeros(0),
        c0=np.array([s.c0 for s in shapes], float),
        rs=np.array([s.rs for s in shapes], float),
        volume=np.array([s.volume for s in shapes], float),
        mass=np.array([s.volume for s in shapes], float) * rho_p,
        inertia=(np.stack([s.inertia_unit for s in shapes]) * rho_p[:, None]) if n else np.zeros((0, 3)),
        pos=pos.copy(), quat=quat.copy(),
        vel=np.zeros((n, 3)) if vel is None else np.asarray(vel, float).reshape(n, 3).copy(),
        omega=np.zeros((n, 3)) if omega is None else np.asarray(omega, float).reshape(n, 3).copy(),
        radius=np.array([s.radius for s in shapes], float),
    )
    ps.refresh_world()
    return ps


def prescribed_state(p0: ParticleSet, lat: LatticeSpec, t: float) -> ParticleSet:
    """Particles moving rigidly with their initial (v, omega) for time t:
    x_p(t) = x_p(0) + v t (wrapped into [0, n) on periodic axes) and
    q(t) = exp(omega t / 2) q(0).  Used to replay one trajectory on both the
    GPU path and the oracle."""
    p = p0.copy()
    dims = lat.dims
    for a in range(3):
        p.pos[:, a] = p0.pos[:, a] + p0.vel[:, a] * t
        if lat.periodic[a]:
            p.pos[:, a] = np.mod(p.pos[:, a], dims[a])
    for i in range(p.n):
        w = p0.omega[i]
        ang = np.linalg.norm(w) * t
        if ang > 0:
            ax = w / np.linalg.norm(w)
            dq = np.concatenate([[np.cos(0.5 * ang)], np.sin(0.5 * ang) * ax])
            q = quat_mul(dq, p0.quat[i])
            p.quat[i] = q / np.linalg.norm(q)
    p.refresh_world()
    return p


# ----------------------------------------------------------------------------
# placements and the five workloads
# ----------------------------------------------------------------------------

def _support(shape: Shape, R: np.ndarray, n: np.ndarray, rng) -> float:
    """Extent of the rotated body along unit vector n (sampled)."""
    dirs = rng.normal(size=(4000, 3))
    dirs /= np.linalg.norm(dirs, axis=1)[:, None]
    # radial search of the level set along each direction
    t = np.linspace(0, shape.radius * 1.05, 400)
    X = t[None, :, None] * dirs[:, None, :]
    inside = _field(shape.pts, shape.K, X) >= shape.c0
    last = np.where(inside.any(1), (inside * np.arange(400)).max(1), 0)
    surf = dirs * t[last][:, None]
    return float((surf @ R.T @ n).max())


def _place_random(rng, shapes, quats, dims, periodic, margin, forced_pairs=0,
                  gap_range=(0.2, 1.0)):
    n = len(shapes)
    pos = np.zeros((n, 3))
    placed = []
    L = np.asarray(dims, float)

    def dist(a, b):
        d = a - b
        for ax in range(3):
            if periodic[ax]:
                d[ax] -= L[ax] * np.round(d[ax] / L[ax])
        return np.linalg.norm(d)

    def ok(i, x):
        for ax in range(3):
            if not periodic[ax] and (x[ax] - shapes[i].radius < margin or
                                     x[ax] + shapes[i].radius > L[ax] - 1 - margin):
                return False
        for j in placed:
            if dist(x, pos[j]) < shapes[i].radius + shapes[j].radius + 0.5:
                return False
        return True

    i = 0
    pair_done = 0
    while i < n:
        if pair_done < forced_pairs and i + 1 < n:
            for _ in range(10000):
                x = rng.uniform(0, L)
                if ok(i, x):
                    break
            pos[i] = x
            placed.append(i)
            nvec = rng.normal(size=3)
            nvec /= np.linalg.norm(nvec)
            Ra = quat_to_matrix(quats[i])
            Rb = quat_to_matrix(quats[i + 1])
            ha = _support(shapes[i], Ra, nvec, rng)
            hb = _support(shapes[i + 1], Rb, -nvec, rng)
            gap = rng.uniform(*gap_range)
            xb = x + nvec * (ha + hb + gap)
            for ax in range(3):
                if periodic[ax]:
                    xb[ax] = np.mod(xb[ax], L[ax])
            # the forced partner skips the bounding-sphere test against i
            saved = placed.pop()
            okb = ok(i + 1, xb)
            placed.append(saved)
            if okb:
                pos[i + 1] = xb
                placed.append(i + 1)
                i += 2
                pair_done += 1
                continue
            placed.pop()
            continue
        for _ in range(100000):
            x = rng.uniform(0, L)
            if ok(i, x):
                break
        else:
            raise RuntimeError("placement failed")
        pos[i] = x
        placed.append(i)
        i += 1
    return pos


def config_c1(seed: int = 1):
    """One sphere (d = 10) settling in a closed 40x40x80 box, tau 0.8, density
    ratio 1.5, 500 steps, FP64."""
    rng = np.random.default_rng(seed)
    lat = LatticeSpec(40, 40, 80, (0, 0, 0), tau=0.8)
    sh = sphere_shape(10.0, 0.1)
    pos = np.array([20.0, 20.0, 60.0]) + rng.uniform(-0.5, 0.5, 3)
    ps = make_particles([sh], pos, np.array([1.0, 0, 0, 0]), 1.5)
    meta = dict(name="c1_sphere_40x40x80", steps=500, storage="f64", rho_r=1.5,
                gravity=(0.0, 0.0, -7.2e-4), n_sub=10)
    return lat, ps, meta


def _c2_shape(rng, rs=0.1, samples_per_unit=2.0):
    pts = np.array([[0.0, 0, 0], [1.0, 0, 0], [2.0, 0, 0], [1.0, 0.6, 0]])
    K = rng.uniform(0.5, 1.5, 4) * 0.12
    return metaball_shape(pts, K, rs, length=24.0, axis=np.array([1.0, 0, 0]),
                          samples_per_unit=samples_per_unit)


def config_c2(seed: int = 2):
    """One 4-control-point metaball (about 24 lu long) settling in a closed
    128x128x256 box, tau 0.6, density ratio 2.0, 20k steps, FP32."""
    rng = np.random.default_rng(seed)
    lat = LatticeSpec(128, 128, 256, (0, 0, 0), tau=0.6)
    sh = _c2_shape(rng)
    ps = make_particles([sh], [64.0, 64.0, 200.0], random_quaternion(rng), 2.0)
    meta = dict(name="c2_metaball_128x128x256", steps=20000, storage="f32", rho_r=2.0,
                gravity=(0.0, 0.0, -6e-5), n_sub=10)
    return lat, ps, meta


def _random_blob(rng, n_pts):
    pts = []
    while len(pts) < n_pts:
        x = rng.uniform(-1, 1, 3)
        if np.linalg.norm(x) <= 1.0:
            pts.append(x)
    return np.array(pts), rng.uniform(0.5, 1.5, n_pts) * 0.3


def config_c3(seed: int = 3, n_particles: int = 200, n: int = 256):
    """200 metaballs (2-6 control points, d_eq 8-16) in a 256^3 periodic box
    driven by a fluid body force along x, with DEM contacts."""
    rng = np.random.default_rng(seed)
    lat = LatticeSpec(n, n, n, (1, 1, 1), tau=0.6, body_force=(1e-5, 0.0, 0.0))
    lib = []
    for _ in range(16):
        pts, K = _random_blob(rng, int(rng.integers(2, 7)))
        lib.append((pts, K))
    shapes = []
    for i in range(n_particles):
        pts, K = lib[i % len(lib)]
        shapes.append(metaball_shape(pts, K, 0.25, d_eq=float(rng.uniform(8, 16)),
                                     samples_per_unit=1.5))
    quats = [random_quaternion(rng) for _ in range(n_particles)]
    pos = _place_random(rng, shapes, quats, lat.dims, lat.periodic, 1.0,
                        forced_pairs=min(10, n_particles // 2))
    ps = make_particles(shapes, pos, np.array(quats), 1.0)
    meta = dict(name="c3_suspension_256cube_200p", steps=2000, storage="f32", rho_r=1.0,
                gravity=(0.0, 0.0, 0.0), n_sub=10)
    return lat, ps, meta


def _surface_cloud(shape: Shape, rng, n_dirs: int = 4000) -> np.ndarray:
    """Body-frame points on the outer surface of the body: along each of
    n_dirs random directions from the centroid, the last sample inside."""
    dirs = rng.normal(size=(n_dirs, 3))
    dirs /= np.linalg.norm(dirs, axis=1)[:, None]
    t = np.linspace(0, shape.radius * 1.05, 400)
    inside = _field(shape.pts, shape.K, t[None, :, None] * dirs[:, None, :]) >= shape.c0
    last = np.where(inside.any(1), (inside * np.arange(400)).max(1), 0)
    return dirs * t[last][:, None]


def _place_lattice(rng, shapes, grid_pos, dims, periodic, jitter, wall_gap=2.5, level=0.8,
                   tries=400):
    """Bodies on jittered lattice sites with random orientations, each drawn
    again (orientation and jitter) until it keeps wall_gap from every wall
    and does not meet a body placed before it: no surface point of one lies
    where the other's field reaches level * c0 (a shell of roughly 10% of
    the radius around each body)."""
    n = len(shapes)
    L = np.asarray(dims, float)
    per = np.asarray([bool(v) for v in periodic])
    clouds = {}
    pos = np.zeros((n, 3))
    quats = np.zeros((n, 4))
    wpts = [None] * n
    radii = np.array([s.radius for s in shapes])

    def field_at(j, X):
        d = X[:, None, :] - wpts[j][None, :, :]
        return (shapes[j].K[None, :] / (d * d).sum(-1)).sum(-1)

    for i in range(n):
        sh = shapes[i]
        if id(sh) not in clouds:
            clouds[id(sh)] = _surface_cloud(sh, rng)
        cloud = clouds[id(sh)]
        for _ in range(tries):
            q = random_quaternion(rng)
            x = grid_pos[i] + rng.uniform(-jitter, jitter, 3)
            R = quat_to_matrix(q[None, :])[0]
            P = cloud @ R.T + x
            fits = True
            for ax in range(3):
                if not per[ax] and (P[:, ax].min() < wall_gap - 0.5 or
                                    P[:, ax].max() > L[ax] - 0.5 - wall_gap):
                    fits = False
            if not fits:
                continue
            W_i = sh.pts @ R.T + x
            D = pos[:i] - x
            D[:, per] -= L[per] * np.round(D[:, per] / L[per])
            near = np.flatnonzero(np.linalg.norm(D, axis=1) <= sh.radius + radii[:i] + 2.0)
            for j in near:
                d = D[j]
                shift = (pos[j] - x) - d          # image of j nearest x
                Pj = clouds[id(shapes[j])] @ quat_to_matrix(quats[j][None, :])[0].T + pos[j] - shift
                wj = wpts[j]
                wpts[j] = wj - shift
                hit = (field_at(j, P) >= level * shapes[j].c0).any()
                wpts[j] = wj
                dd = Pj[:, None, :] - W_i[None, :, :]
                hit = hit or ((sh.K[None, :] / (dd * dd).sum(-1)).sum(-1) >= level * sh.c0).any()
                if hit:
                    fits = False
                    break
            if fits:
                break
        else:
            raise RuntimeError(f"no clear placement for body {i}")
        pos[i], quats[i] = x, q
        wpts[i] = sh.pts @ quat_to_matrix(q[None, :])[0].T + x
    return pos, quats


def config_c4(seed: int = 4, n: int = 512, per_axis: int = 10, storage: str = "f32"):
    """512^3 lattice, periodic in x and y with walls in z, 1000 metaballs at
    20% solids (d_eq ~ 37) on a jittered 10x10x10 lattice, tau 0.55,
    density ratio 1.5, sedimenting.  Orientations and jitters are drawn
    again until every body is clear of the walls and of its neighbours."""
    rng = np.random.default_rng(seed)
    lat = LatticeSpec(n, n, n, (1, 1, 0), tau=0.55)
    npart = per_axis ** 3
    d_eq = (6.0 * 0.2 * n ** 3 / npart / np.pi) ** (1.0 / 3.0)
    lib = []
    for _ in range(8):
        pts, K = _random_blob(rng, int(rng.integers(2, 7)))
        lib.append(metaball_shape(pts, K, 0.25, d_eq=d_eq, samples_per_unit=0.75))
    shapes = [lib[i % len(lib)] for i in range(npart)]
    sp = n / per_axis
    g = (np.arange(per_axis) + 0.5) * sp
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    grid = np.stack([X.ravel(), Y.ravel(), Z.ravel()], -1)
    pos, quats = _place_lattice(rng, shapes, grid, lat.dims, lat.periodic, 0.05 * sp)
    ps = make_particles(shapes, pos, quats, 1.5)
    # treatment bits 1+2+8: at tau 0.55 the extrapolated non-equilibrium part
    # of VIBB for q > 1/2 grows without bound in narrow gaps between
    # neighbouring bodies (plain 1+2 diverges within ~70 steps here)
    meta = dict(name=f"c4_sediment_{n}cube_{npart}p", steps=5000, storage=storage, rho_r=1.5,
                gravity=(0.0, 0.0, -8.8e-6), n_sub=10, treatments=11)
    return lat, ps, meta


def config_c5(seed: int = 5, n: int = 128):
    """128^3 channel (walls in y, periodic x and z), one 4-point metaball at
    prescribed velocity U (|U| <= 0.05), fluid body force along x."""
    rng = np.random.default_rng(seed)
    lat = LatticeSpec(n, n, n, (1, 0, 1), tau=0.6, body_force=(1e-5, 0.0, 0.0))
    sh = _c2_shape(rng)
    # mostly streamwise, so that over 2000 steps the particle drifts at most
    # 15 lattice units towards a wall
    U = np.array([1.0, rng.uniform(-0.15, 0.15), rng.uniform(-0.15, 0.15)])
    U *= rng.uniform(0.02, 0.05) / np.linalg.norm(U)
    ps = make_particles([sh], [n / 2, n / 2, n / 2], random_quaternion(rng), 1.0,
                        vel=U[None, :])
    meta = dict(name="c5_channel_128cube_adjoint", steps=2000, storage="f32", checkpoint=100)
    return lat, ps, meta


def square_metaball(d_eq: float = 14.65, rs: float = 0.1) -> Shape:
    """Flat metaball whose four control points form a square with equal
    weights (K = 0.6 on a unit square, for which the internal body's bounding
    box has a thickness-to-length ratio of 0.845; the paper's shape has
    0.84375), scaled to the volume-equivalent diameter d_eq.  The body frame's
    third axis is the square's normal."""
    pts = np.array([[0.0, 0, 0], [1.0, 0, 0], [0.0, 1, 0], [1.0, 1, 0]])
    return metaball_shape(pts, np.full(4, 0.6), rs, d_eq=d_eq, samples_per_unit=3.0)


def config_dkt(shape: str = "metaball", tau: float | None = None):
    """Two bodies settling one above the other in a closed 150x150x250 box,
    the setting of the paper's two-metaball example (Sec. 4): flat square
    metaballs of the volume of the paper's printed particle (1648 lu^3,
    d_eq = 14.65) or volume-equivalent spheres, centres at heights 220 and
    205 with the lower one 2 lu off the centreline, the squares horizontal;
    density ratio 1200/927; nu = 7.55e-5 m^2/s at dx = 1 mm, dt = 0.2 ms
    (tau = 0.5453); gravity 9.8 m/s^2 = 3.92e-4 lu/step^2; 10 DEM substeps
    per lattice step (dt_DEM = 2e-6 s would be 100).

    The flat faces start 2.3 lu apart, two fluid nodes across.  There, at
    this tau, the VIBB non-equilibrium extrapolation for q > 1/2 grows
    without bound within ~80 steps (FP64 as FP32), so the metaball case
    carries treatment bit 8, which holds that part at its x_f value; the
    spheres run with the reconstruction as printed."""
    if tau is None:
        tau = 0.5 + 3.0 * 7.55e-5 * 2e-4 / 1e-6
    lat = LatticeSpec(150, 150, 250, (0, 0, 0), tau=tau)
    sh = square_metaball() if shape == "metaball" else sphere_shape(14.65, 0.1)
    ps = make_particles([sh, sh], [[75.0, 75.0, 220.0], [77.0, 75.0, 205.0]],
                        [[1.0, 0, 0, 0], [1.0, 0, 0, 0]], 1200.0 / 927.0)
    meta = dict(name=f"dkt_{shape}_150x150x250", steps=7000, storage="f32",
                rho_r=1200.0 / 927.0, gravity=(0.0, 0.0, -3.92e-4), n_sub=10,
                treatments=11 if shape == "metaball" else 3)
    return lat, ps, meta


def config_floor_pair(rho_r: float = 3.0, gap: float = 3.0, tau: float = 0.5453):
    """Two equal spheres (d = 14.65) side by side, `gap` lu apart, released
    0.7 lu above the floor of a closed 48x40x40 box, under relative gravity:
    the setting of the paper's two-sphere test of the near-contact treatments
    (Sec. 3.3), shortened to the phase it is about, the bodies at rest on the
    floor.  A body resting on the floor covers force points below the wall
    plane; with treatment 2 they count with the reference density and the
    resting body feels no net fluid force, without it the fluid pushes it
    into the wall with the reference pressure on the covered patch.  A
    density ratio of 3 keeps the bodies in DEM contact with the floor;
    lighter ones hover one node row above it, where the row's momentum along
    the wall normal flips sign every step without damping and the coupling
    feeds it.  Gaps of one node row between the two spheres behave alike."""
    lat = LatticeSpec(48, 40, 40, (0, 0, 0), tau=tau)
    sh = sphere_shape(14.65, 0.1)
    x0 = 24.0 - (14.65 + gap) / 2
    ps = make_particles([sh, sh], [[x0, 20.2, 8.0], [x0 + 14.65 + gap, 19.9, 8.0]],
                        [[1.0, 0, 0, 0], [1.0, 0, 0, 0]], rho_r)
    meta = dict(name="floor_pair_48x40x40", steps=1500, storage="f64", rho_r=rho_r,
                gravity=(0.0, 0.0, -3.92e-4), n_sub=10, treatments=3)
    return lat, ps, meta


def tiny_case(seed: int, dims=(16, 14, 12), periodic=(1, 0, 1), n_particles=3,
              diameter_range=(3.0, 6.0), tau=0.7, u0=(0.0, 0.0, 0.0),
              speed=0.0, spin=0.0, body_force=(0.0, 0.0, 0.0), allow_near=True):
    """Small lattices (a few thousand nodes) with a handful of metaballs,
    some touching or wrapping across periodic faces; used for bit-exact
    geometry parity and per-step field parity."""
    rng = np.random.default_rng(seed)
    lat = LatticeSpec(*dims, periodic=tuple(periodic), tau=tau, u0=tuple(u0),
                      body_force=tuple(body_force))
    shapes = []
    for i in range(n_particles):
        npts = int(rng.integers(1, 4))
        if npts == 1:
            shapes.append(sphere_shape(float(rng.uniform(*diameter_range)), 0.1))
        else:
            pts, K = _random_blob(rng, npts)
            shapes.append(metaball_shape(pts, K, 0.1, d_eq=float(rng.uniform(*diameter_range)),
                                         samples_per_unit=8.0))
    quats = np.array([random_quaternion(rng) for _ in range(n_particles)])
    L = np.asarray(dims, float)
    pos = np.zeros((n_particles, 3))
    for i in range(n_particles):
        for _ in range(10000):
            x = rng.uniform(0, L)
            good = True
            for a in range(3):
                if not periodic[a]:
                    lo = shapes[i].radius * (0.6 if allow_near else 1.0) - 0.5
                    if x[a] < lo or x[a] > L[a] - 1 - lo:
                        good = False
            for j in range(i):
                d = x - pos[j]
                for a in range(3):
                    if periodic[a]:
                        d[a] -= L[a] * np.round(d[a] / L[a])
                lim = shapes[i].radius + shapes[j].radius
                if np.linalg.norm(d) < (0.7 * lim if allow_near else lim + 1.0):
                    good = False
            if good:
                break
        pos[i] = x
    vel = rng.normal(size=(n_particles, 3)) * speed
    omega = rng.normal(size=(n_particles, 3)) * spin
    ps = make_particles(shapes, pos, quats, 1.5, vel=vel, omega=omega)
    return lat, ps


WORKLOADS = {
    "c1": config_c1,
    "c2": config_c2,
    "c3": config_c3,
    "c4": config_c4,
    "c5": config_c5,
    "dkt_metaball": lambda: config_dkt("metaball"),
    "dkt_sphere": lambda: config_dkt("sphere"),
    "floor_pair": config_floor_pair,
}


def dem_defaults(ps: ParticleSet, gravity=(0.0, 0.0, 0.0), contact_time=20.0, restitution=0.5):
    """Contact constants for a workload (the paper does not give them): a
    linear normal spring whose contact lasts `contact_time` lattice steps for
    the lightest particle, damping for the given restitution, k_t = k_n / 2,
    mu_s = 0.3.  The contact-point Newton iteration stops after 12 steps:
    from the closest pair of control points a pair in contact converges in
    about 4 to 8, and from the previous contact point in 2 or 3; a pair still
    unconverged after 12 (a saddle between bodies far apart) is taken as not
    in contact."""
    m = float(ps.mass.min()) if ps.n else 1.0
    meff = 0.5 * m
    w0 = np.pi / contact_time
    kn = meff * w0 * w0
    lnr = np.log(restitution)
    zeta = -lnr / np.sqrt(np.pi ** 2 + lnr ** 2)
    eta = 2.0 * zeta * np.sqrt(meff * kn)
    return dict(kn=kn, eta_n=eta, kt=0.5 * kn, eta_t=0.0, mu_s=0.3, ctol=1e-3,
                newton_tol=1e-10, newton_iter=12, gravity=tuple(gravity), rho_f=1.0)


# ----------------------------------------------------------------------------
# prescribed trajectories of the drag comparisons against the oracle
# ----------------------------------------------------------------------------

DRAG_CASES = ("c1", "c2", "c3", "c4")


def drag_case(name: str):
    """A replay run on which the force and torque of the GPU path are compared
    with the FP64 oracle: every body moves rigidly with its (v, omega)
    (prescribed_state), so both sides classify the same poses every step.
    Returns (lat, ps0, steps, treatments, description).

      c1  the 40x40x80 sphere moving down at 0.01 lu/step, spinning slowly;
      c2  the 24 lu metaball in the 128x128x256 box descending at about the
          Stokes settling speed while tumbling (2.4 rad over the run);
      c3  the 200 bodies of the 256^3 suspension with seeded velocities;
      c4  the 1000 bodies of the 512^3 sedimentation with seeded velocities,
          with the workload's treatment bits; only short windows of it fit
          the oracle (sub-boxes around sampled bodies)."""
    if name == "c1":
        lat, ps, meta = config_c1()
        ps.vel[:] = [0.0, 0.0, -0.01]
        ps.omega[:] = [0.0, 0.002, 0.0]
        return lat, ps, 200, 3, "c1 40x40x80 sphere d=10, prescribed descent 0.01 lu/step, 200 steps"
    if name == "c2":
        lat, ps, meta = config_c2()
        ps.vel[:] = [0.002, -0.001, -0.015]
        ps.omega[:] = [0.0005, 0.001, -0.0007]
        return (lat, ps, 2000, 3, "c2 128x128x256 metaball 24 lu long, prescribed descent "
                "0.015 lu/step with tumbling, 2000 steps")
    if name == "c3":
        lat, ps, meta = config_c3()
        rng = np.random.default_rng(31)
        ps = ps.copy()
        ps.vel = rng.normal(size=(ps.n, 3)) * 0.01
        ps.omega = rng.normal(size=(ps.n, 3)) * 0.001
        return (lat, ps, 100, int(meta.get("treatments", 3)),
                "c3 256^3 periodic suspension, 200 bodies on prescribed rigid motions, 100 steps")
    if name == "c4":
        lat, ps, meta = config_c4()
        rng = np.random.default_rng(14)
        ps = ps.copy()
        ps.vel = rng.normal(size=(ps.n, 3)) * 0.02
        ps.omega = rng.normal(size=(ps.n, 3)) * 0.001
        return (lat, ps, 3, int(meta["treatments"]),
                "c4 512^3 sedimentation, 1000 bodies on prescribed rigid motions, treatment "
                "bits 1+2+8; sampled bodies over 3 steps")
    raise KeyError(name)


def fingerprint(lat: LatticeSpec, ps: ParticleSet, steps: int, treatments: int) -> str:
    """Short hash of a replay run's inputs, stored with reference results so
    that a change of the inputs is noticed."""
    h = hashlib.sha256()
    h.update(repr((lat.dims, tuple(lat.periodic), float(lat.tau), float(lat.rho0),
                   tuple(map(float, lat.u0)), tuple(map(float, lat.body_force)),
                   int(steps), int(treatments))).encode())
    for k in ("ctrl_off", "body_pts", "K", "c0", "pos", "quat", "vel", "omega"):
        h.update(np.ascontiguousarray(getattr(ps, k)).tobytes())
    return h.hexdigest()[:16]


# ----------------------------------------------------------------------------
# sub-boxes of a large lattice (bounded samples and windowed comparisons)
# ----------------------------------------------------------------------------

def subset(P: ParticleSet, sel, shift) -> ParticleSet:
    """Bodies sel of P (ascending global index), translated by the integer
    vector shift (exact in FP64 for coordinates inside a sub-box)."""
    segs = [np.arange(P.ctrl_off[q], P.ctrl_off[q + 1]) for q in sel]
    ctrl = np.concatenate(segs) if segs else np.zeros(0, int)
    off = np.zeros(len(sel) + 1, np.int32)
    off[1:] = np.cumsum([len(s) for s in segs])
    return ParticleSet(
        ctrl_off=off, body_pts=P.body_pts[ctrl].copy(), K=P.K[ctrl].copy(), c0=P.c0[sel].copy(),
        rs=P.rs[sel].copy(), volume=P.volume[sel].copy(), mass=P.mass[sel].copy(),
        inertia=P.inertia[sel].copy(), pos=P.pos[sel] + shift, quat=P.quat[sel].copy(),
        vel=P.vel[sel].copy(), omega=P.omega[sel].copy(), radius=P.radius[sel].copy(),
        world_pts=P.world_pts[ctrl] + shift)


def bodies_reaching(ps: ParticleSet, lo, hi, pad: float = 2.0):
    """Indices of the bodies whose bounding ball (plus pad) meets [lo, hi)."""
    return [q for q in range(ps.n)
            if all(ps.pos[q, a] + ps.radius[q] + pad >= lo[a] and
                   ps.pos[q, a] - ps.radius[q] - pad <= hi[a] for a in range(3))]


def subbox(lat: LatticeSpec, ps: ParticleSet, lo, hi):
    """The sub-lattice [lo, hi) of lat as a closed box (its faces act as
    walls) with the bodies that reach into it, translated by -lo.  Returns
    (sub-lattice, bodies, their global indices)."""
    lo, hi = np.asarray(lo, int), np.asarray(hi, int)
    wdims = hi - lo
    wlat = LatticeSpec(*map(int, wdims), periodic=(0, 0, 0), tau=lat.tau, rho0=lat.rho0,
                       u0=lat.u0, body_force=lat.body_force)
    near = bodies_reaching(ps, lo, hi)
    return wlat, subset(ps, near, -lo.astype(float)), near
