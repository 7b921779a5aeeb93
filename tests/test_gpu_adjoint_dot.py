"""Dot-product tests of the adjoint, one lattice step at a time.

For one step S and random adjoints of what it produces (lambda_1 for the
populations after it, weights w for its force and torque, and in the coupled
step sigma_1 for the particle state and the contact state after the DEM
call), the adjoint returns J^T applied to them; for a random direction d of
the step's inputs, <J^T (lambda_1, w, ...), d> must equal the directional
derivative of <lambda_1, f_1> + w . (F^h, T^h) + ..., taken by central
differences of the FP64 forward step.  Each case switches on one group of
kernels, so that a transposition error shows up in its own case, along
random directions that the end-to-end objectives do not probe:

  bulk      stream-collide with Guo forcing and the box walls, no particles;
  links     a resting body: the boundary reconstruction (halfway, VIBB, the
            missing-point treatment, the held f^neq) and its force and torque;
  moving    a translating, spinning body: wall velocities, the refill of the
            nodes it uncovers, and the pose through q and the lever arms;
  coupled   a step followed by dem_step with pair and wall contacts: the DEM
            call's adjoint, contact springs and carried contact sums included.
"""
import dataclasses

import numpy as np
import pytest

from paper_2206_11634_amd import binding as B
from paper_2206_11634_amd import workloads as W

pytestmark = pytest.mark.gpu

H = 1e-6


def _lam(gpu, a=None):
    """An adjoint field holding a [Q][ncell] (zeros when None)."""
    lam = gpu.adjoint_field()
    if a is not None:
        cs = int(gpu.sizes.cell_stride)
        lam.view(gpu.Q, cs)[:, :gpu.ncell] = gpu.torch.as_tensor(a, device=gpu.device)
    return lam


def _read(gpu, lam):
    cs = int(gpu.sizes.cell_stride)
    return lam.view(gpu.Q, cs)[:, :gpu.ncell].cpu().numpy()


def _near_equilibrium(lat, rng, Q=19):
    """Populations of a smooth random flow (|u| ~ 0.04, rho 1 +- 0.02) with a
    small non-equilibrium part, so that the collision is nonlinear."""
    from oracle import oracle as O
    x, y, z = np.meshgrid(np.arange(lat.nx), np.arange(lat.ny), np.arange(lat.nz),
                          indexing="ij")
    ph = rng.uniform(0, 2 * np.pi, 6)
    u = np.stack([0.04 * np.sin(2 * np.pi * y / lat.ny + ph[0]),
                  0.03 * np.cos(2 * np.pi * z / lat.nz + ph[1]),
                  0.02 * np.sin(2 * np.pi * x / lat.nx + ph[2])], -1)
    rho = 1.0 + 0.02 * np.sin(2 * np.pi * (x / lat.nx + z / lat.nz) + ph[3])
    # node order x fastest: transpose (x, y, z) -> (z, y, x) before flattening
    flat = lambda a: np.ascontiguousarray(np.transpose(a, (2, 1, 0) + tuple(range(3, a.ndim))))
    rho, u = flat(rho).reshape(-1), flat(u).reshape(-1, 3)
    e, wq, _ = O.stencil(Q)
    cu = u @ e.T.astype(float)                                   # [ncell][Q]
    feq = (wq[None, :] * rho[:, None] * (1 + 3 * cu + 4.5 * cu * cu
                                         - 1.5 * (u * u).sum(1)[:, None])).T
    return feq + 1e-3 * rng.normal(size=feq.shape) * feq


def _dot(a, b):
    return float(np.sum(a * b))


def _assert_dot(adj, fd, what, rtol):
    assert abs(adj - fd) <= rtol * max(abs(fd), 1e-30), (what, adj, fd)
    assert abs(fd) > 0, what


# ---------------------------------------------------------------------------
# one replayed step on a prescribed trajectory (lbm_adjoint)
# ---------------------------------------------------------------------------

class _Replay:
    """One step from state 0 to state 1 of a prescribed trajectory: classify
    at pose 0, step, read the force, classify at pose 1 (the refill)."""

    def __init__(self, lat, ps, treat, states=None, lattice=19):
        self.lat, self.ps, self.treat, self.lattice = lat, ps, treat, lattice
        self.states = states or [W.prescribed_state(ps, lat, 0.0),
                                 W.prescribed_state(ps, lat, 1.0)]

    def run(self, f0, lam1=None, w=None, vel=None, lat=None, states=None, adjoint=False):
        lat = lat or self.lat
        ps, n = self.ps, self.ps.n
        gpu = B.Lattice.for_particles(lat, ps, storage="f64", treatments=self.treat,
                                      lattice=self.lattice)
        try:
            traj = B.DeviceTrajectory(states or self.states,
                                      vel=ps.vel if vel is None else vel)
            gpu.set_populations(f0)
            gpu.classify(traj[0])
            if adjoint:
                gpu.tape_begin(1)
            gpu.step(traj[0])
            F, T = gpu.forces()
            gpu.classify(traj[1])
            if adjoint:
                lam = _lam(gpu, lam1)
                g = gpu.torch.zeros(4 + 3 * n, dtype=gpu.torch.float64, device=gpu.device)
                gx = gpu.torch.zeros((2, max(n, 1), 6), dtype=gpu.torch.float64,
                                     device=gpu.device)
                gpu.adjoint(traj[1], w if w is not None else np.zeros((n, 6)), lam, g, gx)
                return _read(gpu, lam), g.cpu().numpy(), gx[:, :n].cpu().numpy()
            FT = np.concatenate([F.cpu().numpy()[:n], T.cpu().numpy()[:n]], 1)
            return gpu.populations(), FT
        finally:
            gpu.close()

    def owners(self, f0):
        """Owners at pose 0 and at pose 1."""
        gpu = B.Lattice.for_particles(self.lat, self.ps, storage="f64", treatments=self.treat,
                                      lattice=self.lattice)
        traj = B.DeviceTrajectory(self.states, vel=self.ps.vel)
        gpu.set_populations(f0)
        gpu.classify(traj[0])
        o0 = gpu.owner().copy()
        gpu.step(traj[0])
        gpu.classify(traj[1])
        o1 = gpu.owner().copy()
        gpu.close()
        return o0, o1


def _objective(rep, lam1, w, **kw):
    def J(f0):
        f1, FT = rep.run(f0, **kw)
        return _dot(lam1, f1) + _dot(w, FT)
    return J


def _replay_case(rep, f0, seed, rtol, check_pose=False, rtol_pose=1e-6):
    """rtol for the populations, parameters and velocities; rtol_pose for the
    poses, whose step h = 1e-6 stays small enough that no node changes owner
    and whose differences carry ~1e-8 of rounding."""
    rng = np.random.default_rng(seed)
    n = rep.ps.n
    own0, own1 = rep.owners(f0)
    Q = f0.shape[0]
    lam1 = rng.normal(size=(Q, f0.shape[1])) * (own1 == 0)[None, :]
    w = rng.normal(size=(n, 6))
    lam0, g, gx = rep.run(f0, lam1=lam1, w=w, adjoint=True)
    J = _objective(rep, lam1, w)
    # populations
    d = rng.normal(size=f0.shape) * (own0 == 0)[None, :] * f0
    fd = (J(f0 + H * d) - J(f0 - H * d)) / (2 * H)
    _assert_dot(_dot(lam0, d), fd, "populations", rtol)
    # body force (J is a low-order polynomial in F: a large step is exact
    # up to rounding) and tau
    dF = rng.normal(size=3)
    Jp = lambda s: _objective(rep, lam1, w, lat=dataclasses.replace(
        rep.lat, body_force=tuple(np.array(rep.lat.body_force) + s * dF)))(f0)
    _assert_dot(_dot(g[:3], dF), (Jp(1e-4) - Jp(-1e-4)) / 2e-4, "body force", rtol)
    Jt = lambda s: _objective(rep, lam1, w, lat=dataclasses.replace(rep.lat, tau=rep.lat.tau + s))(f0)
    _assert_dot(g[3], (Jt(1e-5) - Jt(-1e-5)) / 2e-5, "tau", rtol)
    if n == 0:
        return
    # wall velocities (the velocities the fluid sees; the poses stay)
    dv = rng.normal(size=(n, 3))
    Jv = lambda s: _objective(rep, lam1, w, vel=rep.ps.vel + s * dv)(f0)
    _assert_dot(_dot(g[4:].reshape(n, 3), dv), (Jv(1e-5) - Jv(-1e-5)) / 2e-5, "velocity", rtol)
    if check_pose:
        # translation of pose k alone (k = 0: links, q, lever arms; k = 1:
        # the refill's lever arm), a small rotation of pose 0
        for k in (0, 1):
            dx = rng.normal(size=(n, 3))

            def Jx(s):
                st = [p.copy() for p in rep.states]
                st[k].pos = st[k].pos + s * dx
                st[k].refresh_world()
                return _objective(rep, lam1, w, states=st)(f0)
            _assert_dot(_dot(gx[k, :, :3], dx), (Jx(H) - Jx(-H)) / (2 * H), f"pose {k}",
                        rtol_pose)
        dth = rng.normal(size=(n, 3))

        def Jr(s):
            st = [p.copy() for p in rep.states]
            for p in range(n):
                a = s * dth[p]
                ang = np.linalg.norm(a)
                dq = np.concatenate([[np.cos(0.5 * ang)], np.sin(0.5 * ang) * a / ang])
                st[0].quat[p] = W.quat_mul(dq, st[0].quat[p])
            st[0].refresh_world()
            return _objective(rep, lam1, w, states=st)(f0)
        _assert_dot(_dot(gx[0, :, 3:], dth), (Jr(H) - Jr(-H)) / (2 * H), "rotation 0",
                    rtol_pose)


@pytest.mark.parametrize("lattice", [19, 15])
def test_dot_product_bulk(lattice):
    """No particles: stream-collide with Guo forcing and halfway walls in y
    (D3Q19, and the paper's D3Q15)."""
    lat = W.LatticeSpec(20, 18, 16, (1, 0, 1), tau=0.62, body_force=(2e-5, 1e-5, -1e-5))
    ps = W.make_particles([], np.zeros((0, 3)), np.zeros((0, 4)), 1.0)
    f0 = _near_equilibrium(lat, np.random.default_rng(1), lattice)
    print(f"dot bulk D3Q{lattice}", flush=True)
    _replay_case(_Replay(lat, ps, 3, lattice=lattice), f0, 11, 1e-7)


def _one_body(vel, omega, seed=2):
    rng = np.random.default_rng(seed)
    lat = W.LatticeSpec(30, 26, 28, (1, 0, 1), tau=0.6, body_force=(1e-5, 0.0, 0.0))
    pts = np.array([[0.0, 0, 0], [1.0, 0, 0], [2.0, 0, 0], [1.0, 0.6, 0]])
    sh = W.metaball_shape(pts, rng.uniform(0.5, 1.5, 4) * 0.12, 0.1, length=10.0,
                          axis=np.array([1.0, 0, 0]), samples_per_unit=4.0)
    sp = W.sphere_shape(7.0, 0.2)
    ps = W.make_particles([sh, sp], [[14.3, 12.7, 13.2], [15.1, 13.4, 22.9]],
                          [W.random_quaternion(rng), [1, 0, 0, 0]], 1.5,
                          vel=np.asarray(vel, float), omega=np.asarray(omega, float))
    return lat, ps


@pytest.mark.parametrize("treat,lattice", [(0, 19), (3, 19), (11, 19), (3, 15)])
def test_dot_product_links_of_a_resting_body(treat, lattice):
    """Two bodies at rest (halfway only 0, VIBB and missing points 3, with
    the held f^neq 11; D3Q15 with 3): the link reconstruction and the force
    and torque weights."""
    lat, ps = _one_body(np.zeros((2, 3)), np.zeros((2, 3)))
    f0 = _near_equilibrium(lat, np.random.default_rng(3), lattice)
    print(f"dot links treat {treat} D3Q{lattice}", flush=True)
    _replay_case(_Replay(lat, ps, treat, lattice=lattice), f0, 20 + treat, 1e-7)


def test_dot_product_moving_bodies_with_refill_and_pose():
    """The bodies translate (about 0.12 lu in the step, so that nodes are
    uncovered and refilled) and spin: wall velocities, refill, and the
    derivatives with respect to each pose."""
    lat, ps = _one_body([[0.12, 0.03, -0.02], [-0.08, 0.05, 0.1]],
                        [[0.01, -0.02, 0.015], [0.0, 0.01, -0.02]])
    f0 = _near_equilibrium(lat, np.random.default_rng(4))
    rep = _Replay(lat, ps, 3)
    o0, o1 = rep.owners(f0)
    assert np.count_nonzero((o0 != 0) & (o1 == 0)) >= 8   # refilled nodes
    print("dot moving", flush=True)
    _replay_case(rep, f0, 30, 1e-7, check_pose=True)


# ---------------------------------------------------------------------------
# one coupled step (lbm_adjoint_coupled): lattice step, dem_step, classify
# ---------------------------------------------------------------------------

SLOTS = 32


def _blob(raw, n):
    """Views into the DEM state: pair records [n][32][8] (active, spring,
    warm start), partner keys [n][32] (partner + 1, 0 free), wall records
    [n][6][8], carried contact sums [n][6]."""
    b = bytearray(raw.tobytes())
    o_key = n * SLOTS * 64
    o_pw = o_key + n * SLOTS * 4
    o_fc = o_pw + n * 6 * 64
    pp = np.frombuffer(b, np.float64, n * SLOTS * 8, 0).reshape(n, SLOTS, 8)
    key = np.frombuffer(b, np.int32, n * SLOTS, o_key).reshape(n, SLOTS)
    pw = np.frombuffer(b, np.float64, n * 48, o_pw).reshape(n, 6, 8)
    fc = np.frombuffer(b, np.float64, n * 6, o_fc).reshape(n, 6)
    return b, pp, key, pw, fc


class _Coupled:
    """A pair of spheres in contact, the lower one pressed onto the wall
    y = -1/2 by gravity, a metaball beside them: a few coupled steps set the
    contacts up (springs and carried contact sums non-zero), then the case is
    the next step."""

    def __init__(self):
        rng = np.random.default_rng(9)
        self.lat = W.LatticeSpec(34, 26, 30, (1, 0, 1), tau=0.7, body_force=(1e-5, 0.0, 0.0))
        sp = W.sphere_shape(8.0, 0.2)
        pts = np.array([[0.0, 0, 0], [1.0, 0, 0], [0.5, 0.8, 0]])
        mb = W.metaball_shape(pts, np.array([0.1, 0.12, 0.08]), 0.1, length=7.0,
                              axis=np.array([1.0, 0, 0]), samples_per_unit=4.0)
        self.ps = W.make_particles(
            [sp, sp, mb], [[12.13, 3.47, 15.21], [12.61, 11.43, 15.52], [24.3, 12.2, 14.1]],
            [[1, 0, 0, 0], [1, 0, 0, 0], W.random_quaternion(rng)], 2.0,
            vel=np.array([[0.02, -0.002, 0.004], [-0.01, -0.03, 0.006], [0.01, 0.0, -0.004]]),
            omega=np.array([[0.0, 0.001, 0.002], [0.003, 0.0, -0.001], [0.002, 0.0, -0.001]]))
        self.n_sub, self.dt = 10, 0.1
        self.prm = B.DemParams.make(**W.dem_defaults(self.ps, gravity=(0.0, -2e-4, 0.0)))
        gpu = B.Lattice.for_particles(self.lat, self.ps, storage="f64")
        parts = B.DeviceParticles(self.ps)
        gpu.classify(parts)
        for _ in range(4):
            gpu.step(parts)
            gpu.forces()
            gpu.dem(parts, self.n_sub, self.dt, self.prm)
            gpu.classify(parts)
        self.ck = gpu.checkpoint().clone()
        self.f0 = gpu.populations()
        self.dem0 = gpu.dem_checkpoint().cpu().numpy().copy()
        self.p0 = parts.to_host(self.ps)
        gpu.close()

    def run(self, s0, dem0, f0, lam1=None, w=None, sig1=None, sc1=None, key1=None,
            adjoint=False):
        """One coupled step from the populations f0 (the moment plane
        recomputed from them), the particle state s0 and the DEM state dem0."""
        n = self.ps.n
        gpu = B.Lattice.for_particles(self.lat, self.ps, storage="f64")
        try:
            parts = B.DeviceParticles(s0)
            gpu.restore(self.ck)
            gpu.set_populations(f0)
            gpu.dem_restore(gpu.torch.as_tensor(dem0, device=gpu.device))
            gpu.classify(parts)
            if adjoint:
                gpu.tape_begin(1)
            gpu.step(parts)
            F, T = gpu.forces()
            FT = np.concatenate([F.cpu().numpy()[:n], T.cpu().numpy()[:n]], 1)
            gpu.dem(parts, self.n_sub, self.dt, self.prm)
            gpu.classify(parts)
            if adjoint:
                lam = _lam(gpu, lam1)
                g = gpu.torch.zeros(4, dtype=gpu.torch.float64, device=gpu.device)
                sig = gpu.torch.as_tensor(sig1.copy(), device=gpu.device)
                # sc1 holds pair springs by the slots of key1: move them to
                # the slots this run's records took (slots are claimed in
                # thread order)
                k_now = _blob(gpu.dem_checkpoint().cpu().numpy(), n)[2]
                scm = sc1.copy()
                scm[:, 6:102] = 0.0
                for p in range(n):
                    for s in range(SLOTS):
                        if key1[p, s] > 0:
                            t = int(np.nonzero(k_now[p] == key1[p, s])[0][0])
                            scm[p, 6 + 3 * t:9 + 3 * t] = sc1[p, 6 + 3 * s:9 + 3 * s]
                sc = gpu.torch.as_tensor(scm.reshape(-1), device=gpu.device)
                gpu.adjoint_coupled(parts, w, self.prm, self.n_sub, self.dt, lam, g, sig, sc)
                return (_read(gpu, lam), g.cpu().numpy(), sig.cpu().numpy(),
                        sc.cpu().numpy().reshape(n, -1))
            return (gpu.populations(), FT, parts.to_host(self.ps),
                    gpu.dem_checkpoint().cpu().numpy(), gpu.owner().copy())
        finally:
            gpu.close()


def _rotvec(qa, qb):
    """theta with qa = exp(theta / 2) qb, to first order: 2 vec(qa conj(qb))."""
    qc = qb * np.array([1.0, -1.0, -1.0, -1.0])
    return np.stack([2.0 * W.quat_mul(qa[i], qc[i])[1:] for i in range(len(qa))])


def _shift_state(p0, d):
    """The state moved by d [n][12] = (x, theta, v, omega)."""
    p = p0.copy()
    p.pos = p0.pos + d[:, 0:3]
    p.vel = p0.vel + d[:, 6:9]
    p.omega = p0.omega + d[:, 9:12]
    for i in range(p.n):
        a = d[i, 3:6]
        ang = np.linalg.norm(a)
        if ang > 0:
            dq = np.concatenate([[np.cos(0.5 * ang)], np.sin(0.5 * ang) * a / ang])
            p.quat[i] = W.quat_mul(dq, p0.quat[i])
    p.refresh_world()
    return p


def test_dot_product_coupled_step_with_contacts():
    """The coupled step in the middle of a pair contact and a wall contact:
    <J^T (lambda_1, w, sigma_1, sigma_c1), d> against differences of the
    forward step along random directions of the populations, of the
    particle state (x, theta, v, omega) and of the contact state (the
    springs of the active pair and wall records, the carried contact sums)."""
    case = _Coupled()
    n = case.ps.n
    rng = np.random.default_rng(41)
    f0 = case.f0
    _, pp0, key0, pw0, fc0 = _blob(case.dem0, n)
    assert np.count_nonzero(key0) >= 1 and np.count_nonzero(pw0[:, :, 0]) >= 1
    assert np.abs(fc0).max() > 0
    f1n, _, s1n, dem1n, own1 = case.run(case.p0, case.dem0, f0)
    _, pp1, key1, pw1, _ = _blob(dem1n, n)
    # random adjoints of the step's results
    lam1 = rng.normal(size=f1n.shape) * (own1 == 0)[None, :]
    w = rng.normal(size=(n, 6))
    sig1 = rng.normal(size=(n, 12))
    sc1 = np.zeros((n, 120))
    sc1[:, 0:6] = rng.normal(size=(n, 6))
    for p in range(n):
        for s in range(SLOTS):
            if key1[p, s] > 0:
                sc1[p, 6 + 3 * s:9 + 3 * s] = rng.normal(size=3)
        for k in range(6):
            if pw1[p, k, 0] != 0:
                sc1[p, 102 + 3 * k:105 + 3 * k] = rng.normal(size=3)
    lam0, g, sig0, sc0 = case.run(case.p0, case.dem0, f0, lam1=lam1, w=w, sig1=sig1, sc1=sc1,
                                  key1=key1, adjoint=True)

    def J(s0, dem0, f=f0):
        f1, FT, s1, dem1, _ = case.run(s0, dem0, f)
        _, p1, k1, w1, c1 = _blob(dem1, n)
        st = np.concatenate([s1.pos - s1n.pos, _rotvec(s1.quat, s1n.quat), s1.vel, s1.omega], 1)
        val = _dot(lam1, f1) + _dot(w, FT) + _dot(sig1, st) + _dot(sc1[:, 0:6], c1)
        # pair springs by partner, against the slots of the unperturbed run
        for p in range(n):
            slot_of = {int(k1[p, s]): s for s in range(SLOTS) if k1[p, s] > 0}
            for s in range(SLOTS):
                if key1[p, s] > 0:
                    val += _dot(sc1[p, 6 + 3 * s:9 + 3 * s], p1[p, slot_of[int(key1[p, s])], 1:4])
            val += _dot(sc1[p, 102:120].reshape(6, 3), w1[p, :, 1:4])
        return val

    # the particle state
    d = rng.normal(size=(n, 12))
    fd = (J(_shift_state(case.p0, H * d), case.dem0) -
          J(_shift_state(case.p0, -H * d), case.dem0)) / (2 * H)
    _assert_dot(_dot(sig0, d), fd, "particle state", 1e-6)
    # the contact state: springs of active records, carried sums
    dc = np.zeros((n, 120))
    dc[:, 0:6] = rng.normal(size=(n, 6))
    for p in range(n):
        for s in range(SLOTS):
            if key0[p, s] > 0:
                dc[p, 6 + 3 * s:9 + 3 * s] = rng.normal(size=3)
        for k in range(6):
            if pw0[p, k, 0] != 0:
                dc[p, 102 + 3 * k:105 + 3 * k] = rng.normal(size=3)

    def moved(s):
        b, pp, key, pw, fc = _blob(case.dem0, n)
        pp = pp.copy()
        pw = pw.copy()
        fc = fc.copy()
        pp[:, :, 1:4] += s * dc[:, 6:102].reshape(n, SLOTS, 3)
        pw[:, :, 1:4] += s * dc[:, 102:120].reshape(n, 6, 3)
        fc += s * dc[:, 0:6]
        out = bytearray(b)
        o_key = n * SLOTS * 64
        o_pw = o_key + n * SLOTS * 4
        o_fc = o_pw + n * 6 * 64
        out[0:o_key] = pp.tobytes()
        out[o_pw:o_fc] = pw.tobytes()
        out[o_fc:o_fc + n * 48] = fc.tobytes()
        return np.frombuffer(bytes(out), np.uint8).copy()
    fd = (J(case.p0, moved(H)) - J(case.p0, moved(-H))) / (2 * H)
    _assert_dot(_dot(sc0, dc), fd, "contact state", 1e-6)
    # the populations at the fluid nodes
    own0 = _owner_at(case, f0)
    d = np.random.default_rng(43).normal(size=f0.shape) * (own0 == 0)[None, :] * f0
    fd = (J(case.p0, case.dem0, f0 + H * d) - J(case.p0, case.dem0, f0 - H * d)) / (2 * H)
    _assert_dot(_dot(lam0, d), fd, "populations", 1e-6)


def _owner_at(case, f0):
    gpu = B.Lattice.for_particles(case.lat, case.ps, storage="f64")
    parts = B.DeviceParticles(case.p0)
    gpu.restore(case.ck)
    gpu.set_populations(f0)
    gpu.classify(parts)
    own = gpu.owner().copy()
    gpu.close()
    return own
