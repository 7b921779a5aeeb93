"""Pins of the oracle's metaball DEM (Sec. 2.1) against textbook closed forms:
ballistic flight, torque-free rotation invariants, and the restitution
coefficient of a linear spring-dashpot contact."""
import numpy as np

from oracle import oracle as O
from paper_2206_11634_amd import workloads as W


def _dem(ps, lat):
    return O.OracleDEM(ps, lat)


def test_free_flight_with_relative_gravity_and_constant_hydro_force():
    """Velocity Verlet is exact for a constant acceleration
    a = (F_h + (m - rho_f V) g) / m."""
    lat = W.LatticeSpec(64, 64, 64, (1, 1, 1))
    ps = W.make_particles([W.sphere_shape(10.0, 0.2)], [30.2, 31.1, 29.7], [1, 0, 0, 0], 1.5,
                          vel=np.array([[0.01, -0.02, 0.005]]))
    x0, v0 = ps.pos.copy(), ps.vel.copy()
    prm = O.DemParams(gravity=(0.0, 0.0, -1e-3), rho_f=1.0)
    Fh = np.array([[0.05, 0.0, -0.02]])
    Th = np.zeros((1, 3))
    dem = _dem(ps, lat)
    t = 0.0
    for _ in range(25):
        dem.step(ps, Fh, Th, prm, n_sub=4, dt=0.25)
        t += 1.0
    m, V = ps.mass[0], ps.volume[0]
    a = (Fh[0] + (m - V) * np.array([0.0, 0.0, -1e-3])) / m
    expect = x0[0] + v0[0] * t + 0.5 * a * t * t
    assert np.allclose(ps.pos[0], expect, rtol=0, atol=1e-11)
    assert np.allclose(ps.vel[0], v0[0] + a * t, rtol=0, atol=1e-13)


def _rotation_drift(n_sub, dt, steps):
    lat = W.LatticeSpec(64, 64, 64, (1, 1, 1))
    rng = np.random.default_rng(4)
    pts = np.array([[0.0, 0, 0], [1.0, 0, 0], [2.0, 0.3, 0], [1.0, 0.8, 0.2]])
    K = rng.uniform(0.5, 1.5, 4) * 0.12
    sh = W.metaball_shape(pts, K, 0.1, length=16.0, axis=np.array([1.0, 0, 0]))
    ps = W.make_particles([sh], [32.0, 32.0, 32.0], W.random_quaternion(rng), 1.0,
                          omega=np.array([[0.05, 0.02, -0.035]]))
    I = ps.inertia[0]

    def invariants():
        R = W.quat_to_matrix(ps.quat[0])
        wb = R.T @ ps.omega[0]
        return 0.5 * (I * wb * wb).sum(), R @ (I * wb)

    E0, L0 = invariants()
    dem = _dem(ps, lat)
    z = np.zeros((1, 3))
    for _ in range(steps):
        dem.step(ps, z, z, O.DemParams(), n_sub=n_sub, dt=dt)
    E1, L1 = invariants()
    assert abs(np.linalg.norm(ps.quat[0]) - 1) < 1e-14
    return abs(E1 - E0) / E0, np.linalg.norm(L1 - L0) / np.linalg.norm(L0)


def test_torque_free_rotation_conserves_energy_and_angular_momentum():
    """Euler's equations without torque keep the kinetic energy and the world
    angular momentum; the integrator's drift falls about fourfold per halving
    of the substep (second order)."""
    e1, l1 = _rotation_drift(2, 0.5, 200)
    e2, l2 = _rotation_drift(4, 0.25, 200)
    assert e1 < 1e-3 and l1 < 1e-3
    assert 3.0 < l1 / l2 < 5.0, (l1, l2)


def _clamped_restitution(zeta):
    """Restitution of m x'' = -k x - eta x' when the contact ends as soon as the
    force k x + eta x' reaches zero (no attraction); Schwager & Poeschel's
    closed form with omega_0 = 1, beta = zeta, omega = sqrt(1 - zeta^2)."""
    b, w = zeta, np.sqrt(1 - zeta ** 2)
    tc = (np.pi - np.arctan2(2 * b * w, w * w - b * b)) / w
    return -np.exp(-b * tc) * (np.cos(w * tc) - (b / w) * np.sin(w * tc))


def test_clamped_restitution_formula_reduces_to_textbook_for_weak_damping():
    z = 1e-3
    assert abs(_clamped_restitution(z) - np.exp(-z * np.pi / np.sqrt(1 - z * z))) < 1e-5


def test_sphere_wall_restitution_matches_linear_spring_dashpot():
    """A sphere (one control point) hitting a wall at v = 0.01 with overlap
    kept near R_s / 2, where the first-order surface-point estimate of
    Eq. (metawallcp) is close to the exact gap."""
    lat = W.LatticeSpec(64, 64, 64, (1, 1, 0))
    r, rs, v = 5.0, 0.1, 0.01
    ps = W.make_particles([W.sphere_shape(2 * r, rs)], [30.0, 30.0, -0.5 + r + 0.3], [1, 0, 0, 0],
                          1.5, vel=np.array([[0.0, 0.0, -v]]))
    m = ps.mass[0]
    zeta = 0.2
    kn = m * (v / 0.05) ** 2
    eta = 2 * zeta * np.sqrt(m * kn)
    prm = O.DemParams(kn=kn, eta_n=eta, kt=kn / 2, eta_t=0.0, mu_s=0.3)
    dem = _dem(ps, lat)
    z = np.zeros((1, 3))
    for _ in range(120):
        dem.step(ps, z, z, prm, n_sub=20, dt=0.05)
    e = ps.vel[0, 2] / v
    e_expect = _clamped_restitution(zeta)
    assert abs(e - e_expect) / e_expect < 0.025, (e, e_expect)
    assert abs(ps.vel[0, 0]) < 1e-14 and abs(ps.vel[0, 1]) < 1e-14


def test_sphere_sphere_head_on_restitution_and_momentum():
    lat = W.LatticeSpec(96, 64, 64, (1, 1, 1))
    r, rs, v = 5.0, 0.1, 0.01
    shs = [W.sphere_shape(2 * r, rs), W.sphere_shape(2 * r, rs)]
    ps = W.make_particles(shs, [[40.0, 32.0, 32.0], [40.0 + 2 * r + 0.4, 32.0, 32.0]],
                          [[1, 0, 0, 0], [1, 0, 0, 0]], 1.5,
                          vel=np.array([[v, 0, 0], [-v, 0, 0]]))
    meff = 0.5 * ps.mass[0]
    zeta = 0.3
    kn = meff * (2 * v / 0.05) ** 2
    eta = 2 * zeta * np.sqrt(meff * kn)
    prm = O.DemParams(kn=kn, eta_n=eta, kt=kn / 2, eta_t=0.0, mu_s=0.3)
    dem = _dem(ps, lat)
    z = np.zeros((2, 3))
    for _ in range(120):
        dem.step(ps, z, z, prm, n_sub=20, dt=0.05)
        assert abs((ps.mass[:, None] * ps.vel).sum(0)).max() < 1e-13
    e = (ps.vel[1, 0] - ps.vel[0, 0]) / (2 * v)
    e_expect = _clamped_restitution(zeta)
    assert abs(e - e_expect) / e_expect < 0.025, (e, e_expect)
    assert np.abs(ps.omega).max() < 1e-14


def test_metaball_pair_contact_is_symmetric():
    """Equal and opposite contact forces for two non-spherical bodies pressed
    together (Newton's third law through the shared contact point)."""
    lat = W.LatticeSpec(96, 64, 64, (1, 1, 1))
    rng = np.random.default_rng(9)
    pts, K = np.array([[0.0, 0, 0], [1.0, 0, 0], [0.5, 0.7, 0]]), rng.uniform(0.5, 1.5, 3) * 0.2
    sh = W.metaball_shape(pts, K, 0.5, d_eq=10.0, samples_per_unit=4.0)
    q1, q2 = W.random_quaternion(rng), W.random_quaternion(rng)
    ps = W.make_particles([sh, sh], [[40.0, 32.0, 32.0], [52.0, 32.5, 31.8]], [q1, q2], 1.5,
                          vel=np.array([[0.02, 0, 0], [-0.02, 0, 0]]))
    prm = O.DemParams(kn=3.0, eta_n=5.0, kt=1.5, eta_t=0.0, mu_s=0.3)
    dem = _dem(ps, lat)
    z = np.zeros((2, 3))
    touched = False
    for _ in range(150):
        dem.step(ps, z, z, prm, n_sub=10, dt=0.1)
        P = (ps.mass[:, None] * ps.vel).sum(0)
        assert np.abs(P).max() < 1e-12
        touched |= bool(np.abs(dem.fc).max() > 0)
    assert touched


def test_unequal_spheres_overlap_follows_the_projection_through_internal_contact():
    """Two sphero-spheres of internal radii a = 4 and b = 2 (K = a^2, b^2).  On
    the centre line the stationary point of M_A + M_B sits where
    K_A / rho_A^3 = K_B / rho_B^3, and the projection of Eq. k0 moves it by
    (1 - K/rho^2) rho^3 / (2K) towards each centre, so the overlap is
    R_sA + R_sB - s_A - s_B in closed form.  The stationary point enters the
    larger internal sphere (rho_A < a) before the internal spheres touch;
    the force must follow the closed form there too (the signed separation)
    and grow monotonically as the centres approach."""
    lat = W.LatticeSpec(64, 64, 64, (1, 1, 1))
    rs = 0.25
    a, b = 4.0, 2.0
    shs = [W.sphere_shape(2 * (a + rs), rs), W.sphere_shape(2 * (b + rs), rs)]
    kn = 2.0
    prm = O.DemParams(kn=kn, eta_n=0.0, kt=1.0, eta_t=0.0, mu_s=0.3, newton_iter=60)
    r = (a * a / (b * b)) ** (1.0 / 3.0)
    seen_inside, last = False, 0.0
    for d in np.linspace(a + b + 0.45, a + b - 0.2, 14):
        ps = W.make_particles(shs, [[30.0, 32.0, 32.0], [30.0 + d, 32.0, 32.0]],
                              [[1, 0, 0, 0], [1, 0, 0, 0]], 1.5)
        dem = _dem(ps, lat)
        z = np.zeros((2, 3))
        dem.step(ps, z, z, prm, n_sub=1, dt=1e-9)
        rho_a = d * r / (1 + r)
        rho_b = d - rho_a
        s_a = (1 - a * a / rho_a ** 2) * rho_a ** 3 / (2 * a * a)
        s_b = (1 - b * b / rho_b ** 2) * rho_b ** 3 / (2 * b * b)
        delta = 2 * rs - s_a - s_b
        seen_inside |= rho_a < a
        f = -dem.fc[0, 0]
        assert abs(dem.fc[0, 1]) < 1e-12 and abs(dem.fc[0, 2]) < 1e-12
        if delta <= 0:
            assert f == 0.0, d
            continue
        assert abs(f - kn * delta) < 1e-9 * kn, (d, f, kn * delta)
        assert f > last
        last = f
    assert seen_inside and last > 0


def test_tilted_flat_metaballs_collide_and_separate():
    """Two flat square metaballs, the lower tilted 0.6 rad and 4 lu off axis,
    approach at 0.005 lu/step.  Their gap is a wedge; the stationary point
    of M_A + M_B enters one internal body before the faces touch.  The
    contact is found, momentum is conserved, and the bodies separate."""
    lat = W.LatticeSpec(150, 150, 250, (0, 0, 0))
    sh = W.square_metaball()
    ang = 0.6
    ps = W.make_particles([sh, sh], [[75.0, 75.0, 120.0], [79.0, 75.0, 104.5]],
                          [[1.0, 0, 0, 0], [np.cos(ang / 2), 0, np.sin(ang / 2), 0]], 1.3,
                          vel=np.array([[0, 0, -0.005], [0, 0, 0]]))
    kw = W.dem_defaults(ps)
    dem = _dem(ps, lat)
    p0 = (ps.mass[:, None] * ps.vel).sum(0)
    z = np.zeros((2, 3))
    touched = 0
    for _ in range(1500):
        dem.step(ps, z, z, O.DemParams(**kw), 10, 0.1)
        touched += bool(np.abs(dem.fc).max() > 0)
        assert np.abs((ps.mass[:, None] * ps.vel).sum(0) - p0).max() < 1e-12
    assert touched > 10
    assert ps.vel[0, 2] > ps.vel[1, 2]           # moving apart along the line of approach
    assert ps.pos[0, 2] - ps.pos[1, 2] > 12.0    # flat faces never passed into each other
