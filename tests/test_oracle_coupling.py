"""Pins of the oracle's coupling physics (Secs. 2.3.1-2.3.5): VIBB, momentum
exchange, refilling and the near-contact treatments, against invariants and
classical Stokes-flow results."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2206_11634_amd import workloads as W
from paper_2206_11634_amd.workloads import Shape

E19 = np.array([(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
                (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1),
                (1, 0, -1), (-1, 0, 1), (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)], float)
W19 = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)


def _feq(i, rho, u):
    eu = E19[i] @ u
    return W19[i] * rho * (1 + 3 * eu + 4.5 * eu * eu - 1.5 * (u @ u))


def _ball(r, pos, omega=None, vel=None):
    sh = Shape(pts=np.zeros((1, 3)), K=np.array([r * r]), c0=1.0, rs=0.0,
               volume=4 / 3 * np.pi * r ** 3, inertia_unit=np.ones(3), radius=r)
    return W.make_particles([sh], pos, [1, 0, 0, 0], 1.0,
                            omega=None if omega is None else np.asarray(omega)[None],
                            vel=None if vel is None else np.asarray(vel)[None])


def test_vibb_matches_geometric_interpolation():
    """The closed-form VIBB coefficients are the linear inter/extrapolation,
    at the departure point x_d = 2q - 1 (x_ff at -1, x_f at 0, wall at q), of
    rho, u and fneq; u_d blends the two velocity estimates 1/3 : 2/3."""
    rng = np.random.default_rng(0)
    for _ in range(200):
        d = int(rng.integers(1, 19))
        db = d + 1 if d % 2 == 1 else d - 1
        q = float(rng.uniform(0.01, 1.0))
        rho_f, rho_ff = rng.uniform(0.95, 1.05, 2)
        u_f, u_ff, uw = (rng.uniform(-0.05, 0.05, 3) for _ in range(3))
        fd_f = _feq(d, rho_f, u_f) * (1 + 0.01 * rng.standard_normal())
        fd_ff = _feq(d, rho_ff, u_ff) * (1 + 0.01 * rng.standard_normal())
        xd = 2 * q - 1
        if xd <= 0:
            ustar = np.array([np.interp(xd, [-1, 0], [u_ff[a], u_f[a]]) for a in range(3)])
            rho_d = np.interp(xd, [-1, 0], [rho_ff, rho_f])
        else:
            ustar = np.array([np.interp(xd, [0, q], [u_f[a], uw[a]]) for a in range(3)])
            rho_d = rho_f
        u2 = np.array([np.interp(xd, [-1, q], [u_ff[a], uw[a]]) for a in range(3)])
        ud = ustar / 3 + 2 * u2 / 3
        line = np.polyfit([-1.0, 0.0], [fd_ff - _feq(d, rho_ff, u_ff), fd_f - _feq(d, rho_f, u_f)], 1)
        fneq = np.polyval(line, xd)
        expect = _feq(d, rho_d, ud) + fneq + 6 * W19[d] * rho_f * (E19[db] @ uw)
        got = O.vibb(d, q, fd_f, rho_f, u_f, fd_ff, rho_ff, u_ff, uw)
        assert abs(got - expect) < 1e-14, (d, q)


def test_vibb_neq_split_is_zeroth_order_beyond_x_f():
    """With treatment bit 8 the departure point's non-equilibrium part for
    x_d beyond x_f (q > 1/2) is held at its x_f value, as rho_d already is;
    for q <= 1/2 nothing changes, and the value no longer depends on f at x_ff."""
    rng = np.random.default_rng(1)
    for _ in range(200):
        d = int(rng.integers(1, 19))
        db = d + 1 if d % 2 == 1 else d - 1
        q = float(rng.uniform(0.01, 1.0))
        rho_f, rho_ff = rng.uniform(0.95, 1.05, 2)
        u_f, u_ff, uw = (rng.uniform(-0.05, 0.05, 3) for _ in range(3))
        fd_f = _feq(d, rho_f, u_f) * (1 + 0.01 * rng.standard_normal())
        fd_ff = _feq(d, rho_ff, u_ff) * (1 + 0.01 * rng.standard_normal())
        lit = O.vibb(d, q, fd_f, rho_f, u_f, fd_ff, rho_ff, u_ff, uw)
        got = O.vibb(d, q, fd_f, rho_f, u_f, fd_ff, rho_ff, u_ff, uw, treat=O.TREAT_NEQ_SPLIT)
        if q <= 0.5:
            assert got == lit
            continue
        xd = 2 * q - 1
        ustar = np.array([np.interp(xd, [0, q], [u_f[a], uw[a]]) for a in range(3)])
        u2 = np.array([np.interp(xd, [-1, q], [u_ff[a], uw[a]]) for a in range(3)])
        expect = (_feq(d, rho_f, ustar / 3 + 2 * u2 / 3) + fd_f - _feq(d, rho_f, u_f)
                  + 6 * W19[d] * rho_f * (E19[db] @ uw))
        assert abs(got - expect) < 1e-14, (d, q)
        moved = O.vibb(d, q, fd_f, rho_f, u_f, 2 * fd_ff, rho_ff, u_ff, uw,
                       treat=O.TREAT_NEQ_SPLIT)
        assert moved == got


def _flat_pair_gap(treat, steps):
    """Two square metaballs (d_eq 14.65, faces horizontal, half-thickness
    6.35) 15 lu apart settle side by side in a closed 48x48x80 box at
    tau = 0.5453: about two fluid nodes separate the parallel faces."""
    lat = W.LatticeSpec(48, 48, 80, (0, 0, 0), tau=0.5453)
    sh = W.square_metaball()
    ps = W.make_particles([sh, sh], [[24.0, 24.0, 55.0], [26.0, 24.0, 40.0]],
                          [[1.0, 0, 0, 0]] * 2, 1200 / 927)
    kw = W.dem_defaults(ps, gravity=(0, 0, -3.92e-4))
    o, dem = O.Oracle(lat, treat=treat), O.OracleDEM(ps, lat)
    umax = 0.0
    for _ in range(steps):
        o.classify(ps)
        F, T = o.step(ps)
        dem.step(ps, F, T, O.DemParams(**kw), 10, 0.1)
        rho, u = o.moments()
        umax = float(np.abs(u[o.owner == 0]).max())
        if not np.isfinite(umax) or umax > 0.1:
            break
    return umax


def test_neq_extrapolation_in_a_two_node_gap():
    """Eq. (neqd) as printed extrapolates for q > 1/2 with weights up to 2 and
    -1; between the two flat faces at tau near 1/2 that grows without bound
    within 80 steps (the bodies have fallen 0.2 lu).  Holding the
    non-equilibrium part at x_f (treatment bit 8) keeps the same flow bounded
    by the settling speed."""
    base = O.TREAT_VIBB | O.TREAT_MISSING
    assert _flat_pair_gap(base, 90) > 0.1
    assert _flat_pair_gap(base | O.TREAT_NEQ_SPLIT, 150) < 0.01


def test_comoving_particles_leave_uniform_flow_exact():
    """Uniform flow f = feq(1, U) with particles translating at U: VIBB, the
    moving-wall bounce-back and both refilling rules return feq(1, U), so the
    populations stay exact and the momentum-exchange forces vanish."""
    U = np.array([0.03, -0.02, 0.015])
    lat, ps = W.tiny_case(7, dims=(20, 18, 16), periodic=(1, 1, 1), n_particles=2,
                          diameter_range=(4, 6), u0=tuple(U), allow_near=False)
    ps.vel[:] = U
    ps.omega[:] = 0
    o = O.Oracle(lat)
    P = W.prescribed_state(ps, lat, 0.0)
    o.classify(P)
    f0 = o.f[:, 0].copy()
    refilled = 0
    for n in range(40):
        F, T = o.step(P)
        assert np.abs(F).max() < 1e-13
        P = W.prescribed_state(ps, lat, n + 1.0)
        o.classify(P)
        refilled += len(o.refill_nodes)
        fl = o.owner == 0
        assert np.abs(o.f[:, fl] - f0[:, None]).max() < 1e-14
    assert refilled > 20


def test_comoving_pair_in_near_contact_with_moving_missing_points():
    """Two spheres 0.4 lu apart translate together at U through a uniform
    flow f = feq(rho0, U), rho0 = 1.03, with treatments 1 and 2 on.  Lattice
    lines from one body run straight into the other, so each body has
    missing force points (Eqs. fh_s_issue, th_s_issue) whose wall velocity
    is U.  A missing point's term is the moving-wall equilibrium
    feq(rho0, u_w) on both sides; at u_w = U it equals what a fluid link at
    that place would give, so every lattice line through a body still
    contributes equal and opposite terms at its two ends and F = 0 exactly
    per body, through covering and refilling, while halfway and VIBB keep
    the populations at feq(rho0, U)."""
    U = np.array([0.03, -0.02, 0.015])
    rho0 = 1.03
    lat = W.LatticeSpec(26, 22, 20, (1, 1, 1), tau=0.7, rho0=rho0, u0=tuple(U))
    sh_a = Shape(pts=np.zeros((1, 3)), K=np.array([9.0]), c0=1.0, rs=0.0,
                 volume=4 / 3 * np.pi * 27, inertia_unit=np.ones(3), radius=3.0)
    sh_b = Shape(pts=np.zeros((1, 3)), K=np.array([12.25]), c0=1.0, rs=0.0,
                 volume=4 / 3 * np.pi * 3.5 ** 3, inertia_unit=np.ones(3), radius=3.5)
    axis = np.array([1.0, 0.7, 0.4]) / np.linalg.norm([1.0, 0.7, 0.4])
    ca = np.array([9.13, 8.41, 9.27])
    ps = W.make_particles([sh_a, sh_b], [ca, ca + (3.0 + 3.5 + 0.4) * axis],
                          [[1, 0, 0, 0]] * 2, 1.5, vel=np.array([U, U]))
    o = O.Oracle(lat, treat=O.TREAT_VIBB | O.TREAT_MISSING)
    P = W.prescribed_state(ps, lat, 0.0)
    o.classify(P)
    f0 = o.f[:, 0].copy()
    assert abs(f0.sum() - rho0) < 1e-14
    missing, refilled, halfway = [0, 0], 0, 0
    for n in range(40):
        kinds = np.bincount(o.links.kind, minlength=3)
        halfway += kinds[O.KIND_HALFWAY]
        for p in range(2):
            missing[p] += int(((o.links.kind == O.KIND_MISSING) & (o.links.part == p)).sum())
        F, T = o.step(P)
        assert np.abs(F).max() < 1e-12, (n, F)
        P = W.prescribed_state(ps, lat, n + 1.0)
        o.classify(P)
        refilled += len(o.refill_nodes)
        fl = o.owner == 0
        assert np.abs(o.f[:, fl] - f0[:, None]).max() < 1e-14
    assert min(missing) > 40 and refilled > 20 and halfway > 0, (missing, refilled, halfway)


def test_missing_force_points_restore_isotropy_near_wall_and_particle():
    """Particles at rest in fluid at rest, one 0.3 lu from a wall and the other
    0.4 lu above it: with treatment 2 every lattice line through a body enters
    and leaves it once, so F = T = 0 to rounding; without it the wall side
    loses force points and a spurious force appears."""
    sh1, sh2 = W.sphere_shape(8.0, 0.1), W.sphere_shape(7.0, 0.1)
    lat = W.LatticeSpec(24, 20, 20, (1, 1, 0), tau=0.7)
    pos = np.array([[10.2, 9.7, -0.5 + 4 + 0.3], [10.6, 9.9, 3.8 + 4 + 3.5 + 0.4]])
    ps = W.make_particles([sh1, sh2], pos, np.array([[1, 0, 0, 0], [1, 0, 0, 0.]]), 1.5)
    o = O.Oracle(lat, treat=O.TREAT_VIBB | O.TREAT_MISSING)
    o.classify(ps)
    assert np.all(np.bincount(o.links.kind, minlength=3) > 0)
    F, T = o.step(ps)
    assert np.abs(F).max() < 1e-13 and np.abs(T).max() < 1e-13
    o2 = O.Oracle(lat, treat=O.TREAT_VIBB)
    o2.classify(ps)
    F2, _ = o2.step(ps)
    assert np.abs(F2).max() > 0.1


@pytest.mark.slow
def test_hasimoto_drag_periodic_sphere_array():
    """Fixed sphere (d = 10) in a periodic 32^3 cell driven by a body force:
    drag / (6 pi mu a U) against Hasimoto's periodic-array factor, with U the
    superficial velocity."""
    L, r, tau, g = 32, 5.0, 0.8, 1e-6
    nu = (tau - 0.5) / 3
    phi = 4 / 3 * np.pi * r ** 3 / L ** 3
    K = 1 / (1 - 1.7601 * phi ** (1 / 3) + phi - 1.5593 * phi ** 2 + 3.9799 * phi ** (8 / 3)
             - 3.0734 * phi ** (10 / 3))
    U_guess = g * (L ** 3 - 4 / 3 * np.pi * r ** 3) / (6 * np.pi * nu * r * K)
    lat = W.LatticeSpec(L, L, L, (1, 1, 1), tau=tau, body_force=(g, 0, 0), u0=(U_guess, 0, 0))
    ps = _ball(r, [L / 2 + 0.13, L / 2 - 0.21, L / 2 + 0.07])
    o = O.Oracle(lat)
    o.classify(ps)
    for _ in range(1500):
        F, _ = o.step(ps)
    rho, u = o.moments()
    fl = o.owner == 0
    U = (rho[fl] * u[fl, 0]).sum() / L ** 3
    ratio = F[0, 0] / (6 * np.pi * nu * r * U) / K
    assert abs(ratio - 1) < 0.03, ratio
    assert abs(F[0, 1]) < 1e-3 * F[0, 0] and abs(F[0, 2]) < 1e-3 * F[0, 0]


@pytest.mark.slow
def test_rotating_sphere_stokes_torque():
    """Sphere (d = 10) spinning in place in fluid at rest: torque close to
    Stokes' -8 pi mu a^3 omega (a periodic cell adds about 1-2%)."""
    L, r, tau = 32, 5.0, 0.8
    nu = (tau - 0.5) / 3
    w = np.array([0.0, 0.0, 2e-4])
    lat = W.LatticeSpec(L, L, L, (1, 1, 1), tau=tau)
    ps = _ball(r, [L / 2 + 0.13, L / 2 - 0.21, L / 2 + 0.07], omega=w)
    o = O.Oracle(lat)
    o.classify(ps)
    for _ in range(1000):
        F, T = o.step(ps)
    ratio = T[0, 2] / (-8 * np.pi * nu * r ** 3 * w[2])
    assert 1.0 < ratio < 1.03, ratio
    assert np.abs(T[0, :2]).max() < 1e-3 * abs(T[0, 2])


def _light_sphere_on_the_floor(tau, steps=1500, two_step_force=False):
    """A sphere (d = 14.65, density ratio 1.29) settling onto the floor of a
    closed 48x40x40 box under relative gravity (the floor pair's setting with
    one body), treatments 1 + 2, the oracle's coupled loop.  With
    two_step_force the DEM is handed the mean of the last two steps' forces
    (a diagnosis, not the method).  Returns the lowest height, the rise after
    it and the largest step-to-step change of the vertical fluid force, in
    units of the submerged weight W."""
    lat = W.LatticeSpec(48, 40, 40, (0, 0, 0), tau=tau)
    ps = W.make_particles([W.sphere_shape(14.65, 0.1)], [[24.0, 20.2, 8.0]], [[1.0, 0, 0, 0]],
                          1.29)
    o = O.Oracle(lat, treat=3)
    dem = O.OracleDEM(ps, lat)
    prm = O.DemParams(**W.dem_defaults(ps, gravity=(0.0, 0.0, -3.92e-4)))
    Wsub = (ps.mass[0] - ps.volume[0]) * 3.92e-4
    z, F, prev = [], [], None
    for _ in range(steps):
        o.classify(ps)
        Fh, Th = o.step(ps)
        Fd = Fh if (not two_step_force or prev is None) else 0.5 * (Fh + prev)
        prev = Fh.copy()
        dem.step(ps, Fd, Th, prm, 10, 0.1)
        z.append(ps.pos[0, 2])
        F.append(Fh[0, 2] / Wsub)
    z, F = np.array(z), np.array(F)
    k = int(np.argmin(z))
    return z.min(), z[k:].max() - z.min(), np.abs(np.diff(F)).max()


@pytest.mark.slow
def test_a_light_body_hops_off_the_floor_by_a_period_two_force_mode_near_tau_one_half():
    """What makes light bodies resting on a wall hop (a property of the
    method, which the oracle shares with the GPU path).  At the paper's tau
    = 0.5453 the light sphere hovers with its lowest point between the wall
    plane and the first node row, and the momentum exchange at the gap's
    links alternates in sign from step to step (BGK over-relaxation: the
    non-equilibrium part flips sign with factor 1 - 1/tau = -0.83 per step)
    with growing amplitude, fed by the body's own response; its mean lifts
    the body about 1.5 lu.  At tau = 0.8 (factor -0.25) the alternation dies
    out and the sphere settles into wall contact; so it does at tau = 0.5453
    when the DEM is handed the mean of two consecutive steps' forces, which
    cancels the period-two part."""
    zmin, rise, jump = _light_sphere_on_the_floor(0.5453)
    assert rise > 1.0 and jump > 20.0, (zmin, rise, jump)
    zmin, rise, jump = _light_sphere_on_the_floor(0.8)
    assert rise < 0.05 and jump < 1.0, (zmin, rise, jump)
    zmin, rise, jump = _light_sphere_on_the_floor(0.5453, two_step_force=True)
    assert rise < 0.05 and jump < 1.0, (zmin, rise, jump)
