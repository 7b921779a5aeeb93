"""Pins of the oracle's metaball DEM (Sec. 2.1) against textbook closed forms:
ballistic flight, torque-free rotation invariants, and the restitution
coefficient of a linear spring-dashpot contact."""
import numpy as np
import pytest

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


# ---- tangential spring and Coulomb limit (Sec. 2.1.1) ----------------------
#
# A sphere on a flat wall or on another sphere, with the normal force settled
# before the tangential motion starts.  The closed forms below are those of a
# rigid sphere with a point contact: sliding under kinetic friction mu_s N,
# rolling without slip under static friction, and the rolling condition
# v = omega * b at the contact.  They fix the sign and size of the spring, the
# damping and the Coulomb rescale, and the lever arm of the contact torque.

def _floor_sphere(rho=2.0, g=1e-4, delta_eq=0.01, mu=0.3):
    """Sphere d = 10, R_s = 0.1, on the floor of a box periodic in x and y,
    with contact constants that give a settled overlap delta_eq under the
    relative weight and a damping ratio 0.7 in both directions."""
    lat = W.LatticeSpec(64, 64, 64, (1, 1, 0))
    ps = W.make_particles([W.sphere_shape(10.0, 0.1)], [30.0, 30.0, -0.5 + 5.0 - 0.005],
                          [1, 0, 0, 0], rho)
    m = ps.mass[0]
    mrel = m - ps.volume[0]
    kn = mrel * g / delta_eq
    kt = kn / 2
    cst = dict(kn=kn, eta_n=1.4 * np.sqrt(m * kn), kt=kt, eta_t=1.4 * np.sqrt(m * kt), mu_s=mu)
    dem = _dem(ps, lat)
    z = np.zeros((1, 3))
    for _ in range(600):                                    # settle the normal contact
        dem.step(ps, z, z, O.DemParams(gravity=(0, 0, -g), **cst), n_sub=1, dt=0.5)
    assert np.abs(ps.vel).max() < 1e-9
    # lever arm from the centre to the contact point (middle of the overlap
    # below the wall plane z = -1/2)
    Rc = ps.pos[0, 2] + 0.5 + 0.5 * delta_eq
    return ps, dem, cst, m, mrel, ps.inertia[0, 1], Rc


def test_sliding_sphere_decelerates_at_the_coulomb_rate_then_rolls():
    """A sphere launched at v0 without spin slides: kinetic friction mu_s N
    with N the relative weight gives dv/dt = -mu_s (1 - rho_f V/m) g and
    d(omega)/dt = mu_s N R_c / I.  Friction acts at the contact, so the
    angular momentum about the contact line, I omega + m R_c v, is conserved;
    the sliding ends when v = omega R_c, at v = m R_c^2 v0 / (I + m R_c^2),
    5/7 v0 for I = 2/5 m R_c^2, independent of mu_s, k_t and eta_t."""
    g, mu, v0, dt = 1e-4, 0.3, 0.01, 0.5
    ps, dem, cst, m, mrel, I, Rc = _floor_sphere(g=g, mu=mu)
    ps.vel[0, 0] = v0
    prm = O.DemParams(gravity=(0, 0, -g), **cst)
    z = np.zeros((1, 3))
    v, w = [], []
    for _ in range(1200):
        dem.step(ps, z, z, prm, n_sub=1, dt=dt)
        v.append(ps.vel[0, 0])
        w.append(ps.omega[0, 1])
    v, w = np.array(v), np.array(w)
    a_slide = mu * mrel * g / m
    k1, k2 = int(50 / dt) - 1, int(150 / dt) - 1             # inside the sliding phase
    assert abs((v[k1] - v[k2]) / (100 * a_slide) - 1) < 1e-3
    assert abs((w[k2] - w[k1]) / (100 * a_slide * m * Rc / I) - 1) < 1e-3
    v_roll = m * Rc ** 2 * v0 / (I + m * Rc ** 2)
    assert abs(v[-1] / v_roll - 1) < 1e-4, (v[-1], v_roll)
    assert abs(w[-1] * Rc / v[-1] - 1) < 1e-4
    assert abs(v_roll / v0 - 5 / 7) < 2e-3
    assert abs(ps.vel[0, 1]) < 1e-15 and np.abs(ps.omega[0, [0, 2]]).max() < 1e-15


@pytest.mark.parametrize("mu", [0.3, 0.05])
def test_sphere_on_an_incline_rolls_or_slides_by_the_friction_angle(mu):
    """Gravity tilted by 20 degrees against the floor's normal (an incline).
    With tan(20 deg) < mu_s (1 + m R_c^2 / I) the sphere rolls without slip,
    held by the static tangential spring: a = m_rel g sin / (m + I / R_c^2),
    omega = v / R_c.  Below it (mu_s = 0.05) it slides: a = (m_rel g sin -
    mu_s N) / m and d(omega)/dt = mu_s N R_c / I, N = m_rel g cos.  The
    sliding case runs without tangential damping, so the Coulomb-limited
    force comes from the spring alone and the spring length it is reset to
    decides the force's direction at every substep."""
    g, dt, th = 1e-4, 0.5, np.radians(20.0)
    ps, dem, cst, m, mrel, I, Rc = _floor_sphere(g=g, mu=mu)
    if mu < 0.1:
        cst["eta_t"] = 0.0
    prm = O.DemParams(gravity=(g * np.sin(th), 0, -g * np.cos(th)), **cst)
    Rc -= 0.5 * 0.01 * (1 - np.cos(th))                      # overlap under the tilted load
    z = np.zeros((1, 3))
    v, w = [], []
    for _ in range(800):
        dem.step(ps, z, z, prm, n_sub=1, dt=dt)
        v.append(ps.vel[0, 0])
        w.append(ps.omega[0, 1])
    k1, k2 = int(100 / dt) - 1, int(300 / dt) - 1
    a = (v[k2] - v[k1]) / 200
    alpha = (w[k2] - w[k1]) / 200
    N = mrel * g * np.cos(th)
    rolls = np.tan(th) < mu * (1 + m * Rc ** 2 / I)
    assert rolls == (mu == 0.3)
    if rolls:
        a_exp = mrel * g * np.sin(th) / (m + I / Rc ** 2)
        alpha_exp = a_exp / Rc
        assert abs(v[k2] - w[k2] * Rc) < 1e-3 * v[k2]
    else:
        a_exp = (mrel * g * np.sin(th) - mu * N) / m
        alpha_exp = mu * N * Rc / I
        assert v[k2] - w[k2] * Rc > 0.1 * v[k2]
    assert abs(a / a_exp - 1) < 1e-3, (a, a_exp)
    assert abs(alpha / alpha_exp - 1) < 1e-3, (alpha, alpha_exp)


@pytest.mark.parametrize("rolling_index", [0, 1])
def test_sphere_rolling_over_a_fixed_sphere_conserves_energy(rolling_index):
    """A sphere (d = 10) on top of a heavy sphere (d = 16, held against
    gravity by a constant external force), released 0.15 rad from the top
    after its contact has settled under a force equal to gravity's normal
    component.  Rolling without slip, friction does no work and the contact
    normal turns with the body: the kinetic energy gained equals the
    relative weight times the drop (the contact springs' energy counted),
    and the ratio of the centre's tangential speed to omega stays fixed
    (the rolling condition at a fixed lever arm).  Both index orders, so the
    rolling body's spin enters the relative velocity once as body i and once
    as body j."""
    g, dt, th0 = 1e-4, 0.5, 0.15
    lat = W.LatticeSpec(96, 96, 96, (1, 1, 1))
    cA = np.array([48.0, 48.0, 40.0])
    n0 = np.array([np.sin(th0), 0.0, np.cos(th0)])
    big, small = W.sphere_shape(16.0, 0.1), W.sphere_shape(10.0, 0.1)
    order = [small, big] if rolling_index == 0 else [big, small]
    pos = [cA + 12.872 * n0, cA] if rolling_index == 0 else [cA, cA + 12.872 * n0]
    rho = np.array([2.0, 1e9]) if rolling_index == 0 else np.array([1e9, 2.0])
    ps = W.make_particles(order, pos, [[1, 0, 0, 0]] * 2, rho)
    b, h = rolling_index, 1 - rolling_index
    m, I = ps.mass[b], ps.inertia[b, 1]
    mrel = m - ps.volume[b]
    kn = mrel * g / 0.005
    kt = kn / 2
    prm = O.DemParams(kn=kn, eta_n=1.4 * np.sqrt(m * kn), kt=kt, eta_t=1.4 * np.sqrt(m * kt),
                      mu_s=1.0, gravity=(0, 0, -g))
    dem = _dem(ps, lat)
    Fh, Th = np.zeros((2, 3)), np.zeros((2, 3))
    Fh[h, 2] = (ps.mass[h] - ps.volume[h]) * g
    Fh[b] = np.array([0, 0, mrel * g]) - n0 * mrel * g * np.cos(th0)
    for _ in range(600):
        dem.step(ps, Fh, Th, prm, n_sub=1, dt=dt)
    Fh[b] = 0.0

    def state():
        d = ps.pos[b] - ps.pos[h]
        n = d / np.linalg.norm(d)
        fn = dem.fc[b] @ n
        ft = np.linalg.norm(dem.fc[b] - fn * n)
        E = (0.5 * m * ps.vel[b] @ ps.vel[b] + 0.5 * I * ps.omega[b] @ ps.omega[b]
             + mrel * g * ps.pos[b, 2] + fn ** 2 / (2 * kn) + ft ** 2 / (2 * kt))
        vt = ps.vel[b, 0] * n[2] - ps.vel[b, 2] * n[0]
        return np.arctan2(d[0], d[2]), E, vt, ps.omega[b, 1], fn, ft

    _, E0, _, _, _, _ = state()
    z0 = ps.pos[b, 2]
    ratios, dE = [], []
    for k in range(4000):
        dem.step(ps, Fh, Th, prm, n_sub=1, dt=dt)
        th, E, vt, w, fn, ft = state()
        dE.append(abs(E - E0))
        if k > 40:
            assert fn > 0 and ft < fn
        if th > 0.2:
            ratios.append(vt / w)
        if th > 0.7:
            break
    assert th > 0.7
    drop = mrel * g * (z0 - ps.pos[b, 2])
    assert max(dE) < 1e-4 * drop, (max(dE), drop)
    ratios = np.array(ratios)
    assert np.ptp(ratios) < 1e-3 * ratios.mean()
    assert 4.8 < ratios.mean() < 5.0       # the contact point sits inside the sphere's surface
