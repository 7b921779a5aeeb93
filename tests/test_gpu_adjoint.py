"""Adjoint gradients (differentiation form) against central finite
differences of the forward pass and of the FP64 oracle, with the geometry
schedule of the nominal trajectory held fixed."""
import dataclasses

import numpy as np
import pytest

from oracle import oracle as O
from paper_2206_11634_amd import adjoint as AD
from paper_2206_11634_amd import binding as B
from paper_2206_11634_amd import workloads as W

pytestmark = pytest.mark.gpu


def _problem(storage, steps=48, window=20, n=28):
    rng = np.random.default_rng(51)
    lat = W.LatticeSpec(n, n - 4, n, (1, 0, 1), tau=0.7, body_force=(1e-5, 0.0, 0.0))
    pts = np.array([[0.0, 0, 0], [1.0, 0, 0], [2.0, 0, 0], [1.0, 0.6, 0]])
    sh = W.metaball_shape(pts, rng.uniform(0.5, 1.5, 4) * 0.12, 0.1, length=8.0,
                          axis=np.array([1.0, 0, 0]), samples_per_unit=4.0)
    sh2 = W.sphere_shape(6.0, 0.1)
    # particle 1 dips 0.2 lattice units below the wall y = 0 (halfway and
    # missing-point links), clear of particle 0 along z
    ps = W.make_particles([sh, sh2], [[n / 2, (n - 4) / 2, n / 2], [n / 2 + 1.0, 2.8, n / 2 + 9.0]],
                          [W.random_quaternion(rng), [1, 0, 0, 0]], 1.0,
                          vel=np.array([[0.04, 0.006, -0.005], [0.03, 0.0, 0.01]]),
                          omega=np.zeros((2, 3)))
    w = np.zeros((2, 6))
    w[0, 0] = 1.0 / steps
    w[0, 4] = 0.5 / steps
    w[1, 1] = 0.3 / steps
    # initial populations: the fluid at rest, f_i = w_i (D3Q19 numbering: rest,
    # 6 axis directions, 12 face diagonals)
    wq = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
    f0 = np.repeat(wq[:, None], lat.ncell, axis=1)
    return AD.Problem(lat=lat, ps=ps, steps=steps, window=window, storage=storage, weights=w, f0=f0)


def _fd(prob, v, F, tau, which, k, h, fn):
    def at(dv):
        vv, FF, tt = v.copy(), np.array(F, float), tau
        if which == "v":
            vv[k // 3, k % 3] += dv
        elif which == "F":
            FF[k] += dv
        else:
            tt += dv
        return fn(prob, vv, FF, tt)
    return (at(h) - at(-h)) / (2 * h)


def _gpu_J(prob, v, F, tau):
    return AD.evaluate(prob, v, F, tau, grad=False)


def _check(prob, fd_prob, fn, rtol):
    v = prob.ps.vel.copy()
    F = np.array(prob.lat.body_force)
    tau = prob.lat.tau
    J, dv, dF, dtau = AD.evaluate(prob, v, F, tau, grad=True)
    J64 = fn(fd_prob, v, F, tau)
    assert abs(J - J64) <= 1e-4 * abs(J64) + 1e-12
    scale = max(np.abs(dv).max(), 1e-12)
    for k in range(6):
        g = _fd(fd_prob, v, F, tau, "v", k, 1e-5, fn)
        assert abs(dv[k // 3, k % 3] - g) <= rtol * scale, (k, dv[k // 3, k % 3], g)
    gF = _fd(fd_prob, v, F, tau, "F", 0, 1e-6, fn)
    assert abs(dF[0] - gF) <= rtol * abs(gF), (dF[0], gF)
    gt = _fd(fd_prob, v, F, tau, "tau", 0, 1e-5, fn)
    assert abs(dtau - gt) <= rtol * abs(gt), (dtau, gt)
    return dv, dF, dtau


def test_fp64_adjoint_matches_finite_differences():
    prob = _problem("f64")
    _check(prob, prob, _gpu_J, 2e-6)


def test_fp64_adjoint_with_neq_split_matches_finite_differences():
    """Treatment bit 8 changes the VIBB reconstruction for q > 1/2; its
    transpose in the link adjoint follows."""
    prob = dataclasses.replace(_problem("f64"),
                               treatments=B.TREAT_VIBB | B.TREAT_MISSING | B.TREAT_NEQ_SPLIT)
    _check(prob, prob, _gpu_J, 2e-6)


def test_fp32_adjoint_within_1e3_of_fp64_finite_differences():
    prob = _problem("f32")
    _check(prob, dataclasses.replace(prob, storage="f64"), _gpu_J, 1e-3)


def _oracle_J(prob, v, F, tau):
    lat = dataclasses.replace(prob.lat, body_force=tuple(F), tau=tau)
    o = O.Oracle(lat)
    o.f[...] = prob.f0
    def state(n):
        P = W.prescribed_state(prob.ps, prob.lat, float(n))
        P.vel = np.asarray(v, float).copy()
        return P
    o.classify(state(0))
    J = 0.0
    for n in range(prob.steps):
        Fh, Th = o.step(state(n))
        J += float((prob.weights[:, :3] * Fh).sum() + (prob.weights[:, 3:] * Th).sum())
        o.classify(state(n + 1))
    return J


def test_fp64_adjoint_matches_oracle_reference_gradient():
    """The reference gradient is central differences of the FP64 CPU oracle."""
    prob = _problem("f64", steps=30, window=12, n=26)
    _check(prob, prob, _oracle_J, 5e-6)


def test_windowed_recomputation_matches_a_single_window():
    prob = _problem("f64", steps=30, window=7)
    one = dataclasses.replace(prob, window=30)
    v, F, tau = prob.ps.vel.copy(), np.array(prob.lat.body_force), prob.lat.tau
    a = AD.evaluate(prob, v, F, tau, grad=True)
    b = AD.evaluate(one, v, F, tau, grad=True)
    assert abs(a[0] - b[0]) <= 1e-13 * abs(b[0])
    np.testing.assert_allclose(a[1], b[1], rtol=1e-10, atol=1e-12 * np.abs(b[1]).max())
    np.testing.assert_allclose(a[2], b[2], rtol=1e-10)
    # dJ/dtau sums a node-wise product whose terms cancel; atomics add the
    # block partial sums in no fixed order
    assert abs(a[3] - b[3]) <= 1e-7 * abs(b[3])


def test_taping_windows_leave_the_run_unchanged():
    """Taped steps stream through the tape's own buffers; the run's
    populations are bit-identical with and without taping: full and partial
    windows, steps after a full window, an adjoint taken from a partial
    window, a window begun while the last one was never consumed, and
    populations read in the middle of a window."""
    import torch
    prob = _problem("f32", steps=24, window=6)
    states, f0 = prob.states(), prob.initial()

    def run(schedule):
        gpu = B.Lattice.for_particles(prob.lat, prob.ps, storage="f32", treatments=prob.treatments)
        traj = B.DeviceTrajectory(states, vel=prob.ps.vel)
        gpu.set_populations(f0)
        gpu.classify(traj[0])
        seen = []
        for k in range(24):
            act = schedule.get(k)
            if act == "peek":
                seen.append(gpu.populations())
            elif act == "adjoint":
                lam = gpu.adjoint_field()
                g = torch.zeros(4 + 3 * prob.ps.n, dtype=torch.float64, device=gpu.device)
                gpu.adjoint(traj[k], prob.weights, lam, g)
                assert np.isfinite(g.cpu().numpy()).all()
            elif act is not None:
                gpu.tape_begin(act)
            gpu.step(traj[k])
            gpu.classify(traj[k + 1])
        seen.append(gpu.populations())
        gpu.close()
        return seen

    ref = run({5: "peek", 13: "peek"})
    got = run({2: 4, 5: "peek", 8: 7, 11: "adjoint", 13: "peek", 15: 3, 20: 2})
    for a, b in zip(got, ref):
        np.testing.assert_array_equal(a, b)


def test_geometry_snapshots_replay_the_classifications():
    """A replay whose classifications are replaced by the geometry kept from
    the first pass (lbm_geometry_save / lbm_geometry_load: owners, flags,
    links, refilled nodes) has bit-identical populations and owners at every
    step, refills included; a snapshot sized for other list capacities is
    refused with ESTATE."""
    prob = _problem("f32", steps=24, window=6)
    states, f0 = prob.states(), prob.initial()
    gpu = B.Lattice.for_particles(prob.lat, prob.ps, storage="f32", treatments=prob.treatments)
    traj = B.DeviceTrajectory(states, vel=prob.ps.vel)
    gpu.set_populations(f0)
    gpu.classify(traj[0])
    ck = gpu.checkpoint()
    snaps, pops, owners, refills = [gpu.geometry_save()], [], [], 0
    for k in range(24):
        gpu.step(traj[k])
        refills += gpu.classify(traj[k + 1]).n_refill
        snaps.append(gpu.geometry_save())
        pops.append(gpu.populations())
        owners.append(gpu.owner().copy())
    assert refills > 0
    gpu.restore(ck)
    gpu.geometry_load(snaps[0], traj[0])
    for k in range(24):
        gpu.step(traj[k])
        gpu.geometry_load(snaps[k + 1], traj[k + 1])
        np.testing.assert_array_equal(gpu.populations(), pops[k])
        np.testing.assert_array_equal(gpu.owner(), owners[k])
    with pytest.raises(B.LbmError) as e:
        gpu.geometry_load((snaps[0][0], snaps[0][1] ^ 1), traj[0])
    assert e.value.code == B.LBM_ESTATE
    gpu.close()


def test_autograd_function_returns_the_adjoint_gradient():
    import torch
    prob = _problem("f64", steps=20, window=8)
    v = torch.tensor(prob.ps.vel, dtype=torch.float64, requires_grad=True)
    F = torch.tensor(prob.lat.body_force, dtype=torch.float64, requires_grad=True)
    tau = torch.tensor(prob.lat.tau, dtype=torch.float64, requires_grad=True)
    J = AD.DragFunction.apply(v, F, tau, prob)
    (2.0 * J).backward()
    ref = AD.evaluate(prob, prob.ps.vel, np.array(prob.lat.body_force), prob.lat.tau, grad=True)
    assert abs(float(J.detach()) - ref[0]) <= 1e-13 * abs(ref[0])
    np.testing.assert_allclose(v.grad.numpy(), 2 * ref[1], rtol=1e-10, atol=1e-14)
    np.testing.assert_allclose(F.grad.numpy(), 2 * ref[2], rtol=1e-10)
    assert abs(float(tau.grad) - 2 * ref[3]) <= 1e-7 * abs(ref[3])


def _shifted(prob, dx=None, dv=None):
    ps = prob.ps.copy()
    if dx is not None:
        ps.pos = ps.pos + dx
    if dv is not None:
        ps.vel = ps.vel + dv
    ps.refresh_world()
    return dataclasses.replace(prob, ps=ps)


def _geometry_problem(omega):
    prob = _problem("f64", steps=24, window=10)
    ps = prob.ps.copy()
    ps.omega = np.array([[0.0, 0.0, omega], [0.0, 0.0, 0.0]])
    return dataclasses.replace(prob, ps=ps)


@pytest.mark.parametrize("omega", [0.0, 0.004])
def test_fp64_geometry_adjoint_matches_moving_geometry_differences(omega):
    """dJ/dx_p(0) (sum of the pose gradients) against central differences
    that translate the whole trajectory, and the full dJ/dv0 (wall velocity
    and poses together) against differences of v0; both replay the moved
    geometry.  Steps are few and h small so that no owner changes."""
    prob = _geometry_problem(omega)
    v, F, tau = prob.ps.vel.copy(), np.array(prob.lat.body_force), prob.lat.tau
    J, dv, dF, dtau, gx = AD.evaluate(prob, v, F, tau, grad=True, geometry=True)
    gx0, dv0, _ = AD.trajectory_gradients(prob, gx, dv)
    scale = max(np.abs(gx0).max(), 1e-12)
    h = 1e-6
    for p in range(2):
        for a in range(3):
            e = np.zeros((2, 3))
            e[p, a] = h
            Jp = AD.evaluate(_shifted(prob, dx=e), v, F, tau)
            Jm = AD.evaluate(_shifted(prob, dx=-e), v, F, tau)
            fd = (Jp - Jm) / (2 * h)
            assert abs(gx0[p, a] - fd) <= 2e-5 * scale, (p, a, gx0[p, a], fd)
    scale = max(np.abs(dv0).max(), 1e-12)
    for p in range(2):
        for a in range(3):
            e = np.zeros((2, 3))
            e[p, a] = h
            Pp, Pm = _shifted(prob, dv=e), _shifted(prob, dv=-e)
            fd = (AD.evaluate(Pp, v + e, F, tau) - AD.evaluate(Pm, v - e, F, tau)) / (2 * h)
            assert abs(dv0[p, a] - fd) <= 2e-5 * scale, (p, a, dv0[p, a], fd)
    assert np.abs(gx0).max() > 0


def test_fp64_geometry_adjoint_matches_oracle_differences():
    """The reference: central differences of the FP64 oracle's J with the
    whole trajectory translated, its own geometry rebuilt."""
    prob = _geometry_problem(0.004)
    prob = dataclasses.replace(prob, steps=16)
    v, F, tau = prob.ps.vel.copy(), np.array(prob.lat.body_force), prob.lat.tau
    J, dv, dF, dtau, gx = AD.evaluate(prob, v, F, tau, grad=True, geometry=True)
    gx0, _, _ = AD.trajectory_gradients(prob, gx, dv)
    scale = max(np.abs(gx0).max(), 1e-12)
    h = 1e-6
    for p, a in [(0, 0), (0, 2), (1, 1)]:
        e = np.zeros((2, 3))
        e[p, a] = h
        fd = (_oracle_J(_shifted(prob, dx=e), v, F, tau) -
              _oracle_J(_shifted(prob, dx=-e), v, F, tau)) / (2 * h)
        assert abs(gx0[p, a] - fd) <= 5e-5 * scale, (p, a, gx0[p, a], fd)


def test_fp64_geometry_adjoint_with_exact_q():
    prob = dataclasses.replace(_geometry_problem(0.0),
                               treatments=B.TREAT_VIBB | B.TREAT_MISSING | B.TREAT_EXACT_Q)
    v, F, tau = prob.ps.vel.copy(), np.array(prob.lat.body_force), prob.lat.tau
    J, dv, dF, dtau, gx = AD.evaluate(prob, v, F, tau, grad=True, geometry=True)
    gx0, _, _ = AD.trajectory_gradients(prob, gx, dv)
    scale = max(np.abs(gx0).max(), 1e-12)
    h = 1e-6
    for p, a in [(0, 0), (0, 1), (1, 2)]:
        e = np.zeros((2, 3))
        e[p, a] = h
        fd = (AD.evaluate(_shifted(prob, dx=e), v, F, tau) -
              AD.evaluate(_shifted(prob, dx=-e), v, F, tau)) / (2 * h)
        assert abs(gx0[p, a] - fd) <= 2e-5 * scale, (p, a, gx0[p, a], fd)


def _rotated(prob, p, axis, ang):
    ps = prob.ps.copy()
    ax = np.zeros(3)
    ax[axis] = 1.0
    dq = np.concatenate([[np.cos(0.5 * ang)], np.sin(0.5 * ang) * ax])
    ps.quat[p] = W.quat_mul(dq, ps.quat[p])
    ps.refresh_world()
    return dataclasses.replace(prob, ps=ps)


@pytest.mark.parametrize("omega", [0.0, 0.004])
def test_fp64_rotation_adjoint_matches_moving_geometry_differences(omega):
    """dJ/dtheta of the initial orientation (summed over the poses, each
    rotated by the trajectory's own rotation) against central differences
    that rotate the initial quaternion and rebuild the geometry."""
    prob = _geometry_problem(omega)
    v, F, tau = prob.ps.vel.copy(), np.array(prob.lat.body_force), prob.lat.tau
    J, dv, dF, dtau, gx = AD.evaluate(prob, v, F, tau, grad=True, geometry=True)
    _, _, gt0 = AD.trajectory_gradients(prob, gx, dv)
    scale = max(np.abs(gt0[0]).max(), 1e-12)
    h = 1e-6
    for a in range(3):
        fd = (AD.evaluate(_rotated(prob, 0, a, h), v, F, tau) -
              AD.evaluate(_rotated(prob, 0, a, -h), v, F, tau)) / (2 * h)
        assert abs(gt0[0, a] - fd) <= 2e-5 * scale, (a, gt0[0, a], fd)
    assert np.abs(gt0[0]).max() > 0


def test_d3q15_fp64_adjoint_matches_finite_differences():
    """The adjoint kernels built for the paper's D3Q15 lattice."""
    prob = _problem("f64", steps=30, window=12, n=26)
    w15 = np.array([2 / 9] + [1 / 9] * 6 + [1 / 72] * 8)
    f0 = np.repeat(w15[:, None], prob.lat.ncell, axis=1)
    prob = dataclasses.replace(prob, lattice=15, f0=f0)
    _check(prob, prob, _gpu_J, 2e-6)


# ---------------------------------------------------------------------------
# free motion: the adjoint through dem_step
# ---------------------------------------------------------------------------

def _free_problem(steps=20, window=8):
    rng = np.random.default_rng(77)
    n = 30
    lat = W.LatticeSpec(n, n - 2, n, (1, 0, 1), tau=0.7, body_force=(1e-5, 0.0, 0.0))
    pts = np.array([[0.0, 0, 0], [1.0, 0, 0], [2.0, 0, 0], [1.0, 0.6, 0]])
    sh = W.metaball_shape(pts, rng.uniform(0.5, 1.5, 4) * 0.12, 0.1, length=8.0,
                          axis=np.array([1.0, 0, 0]), samples_per_unit=4.0)
    sh2 = W.sphere_shape(6.0, 0.1)
    ps = W.make_particles([sh, sh2], [[n / 2, (n - 2) / 2, n / 2], [n / 2 + 1.0, 7.0, n / 2 + 9.5]],
                          [W.random_quaternion(rng), [1, 0, 0, 0]], 1.5,
                          vel=np.array([[0.03, 0.004, -0.005], [0.02, 0.0, 0.01]]),
                          omega=np.array([[0.002, -0.001, 0.003], [0.0, 0.001, 0.0]]))
    w = np.zeros((2, 6))
    w[0, 0] = 1.0 / steps
    w[0, 4] = 0.5 / steps
    w[1, 1] = 0.3 / steps
    wq = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
    f0 = np.repeat(wq[:, None], lat.ncell, axis=1)
    return AD.FreeProblem(lat=lat, ps=ps, steps=steps, window=window, storage="f64", weights=w,
                          f0=f0, gravity=(0.0, -2e-4, 0.0))


def _free_shift(prob, p, block, a, h):
    ps = prob.ps.copy()
    if block == 0:
        ps.pos[p, a] += h
    elif block == 1:
        ax = np.zeros(3)
        ax[a] = 1.0
        dq = np.concatenate([[np.cos(0.5 * h)], np.sin(0.5 * h) * ax])
        ps.quat[p] = W.quat_mul(dq, ps.quat[p])
    elif block == 2:
        ps.vel[p, a] += h
    else:
        ps.omega[p, a] += h
    ps.refresh_world()
    return dataclasses.replace(prob, ps=ps)


def test_fp64_free_motion_adjoint_matches_finite_differences():
    """dJ/d(x, theta, v, omega) of both initial states, dJ/dF and dJ/dtau of
    a 20-step run in which the DEM moves the bodies under the step's forces
    and gravity (windows of 8), against central differences of the same
    free-motion forward pass, each block within 2e-5 of its largest entry."""
    prob = _free_problem()
    F, tau = np.array(prob.lat.body_force), prob.lat.tau
    J, s0, dF, dtau = AD.evaluate_free(prob, F, tau, grad=True)
    h = 1e-6
    for block in range(4):
        scale = max(np.abs(s0[:, 3 * block:3 * block + 3]).max(), 1e-12)
        for p in range(2):
            for a in range(3):
                fd = (AD.evaluate_free(_free_shift(prob, p, block, a, h), F, tau) -
                      AD.evaluate_free(_free_shift(prob, p, block, a, -h), F, tau)) / (2 * h)
                got = s0[p, 3 * block + a]
                assert abs(got - fd) <= 2e-5 * scale, (block, p, a, got, fd)
    e = np.array([1e-6, 0.0, 0.0])
    fd = (AD.evaluate_free(prob, F + e, tau) - AD.evaluate_free(prob, F - e, tau)) / 2e-6
    assert abs(dF[0] - fd) <= 2e-5 * abs(fd), (dF[0], fd)
    fd = (AD.evaluate_free(prob, F, tau + 1e-6) - AD.evaluate_free(prob, F, tau - 1e-6)) / 2e-6
    assert abs(dtau - fd) <= 2e-5 * abs(fd), (dtau, fd)
    assert np.abs(s0).max() > 0


def test_fp32_free_motion_adjoint_within_1e3_of_fp64_differences():
    """The free-motion adjoint in FP32 storage (FP32 lattice arithmetic, FP64
    DEM and parameter sums) against central differences of the FP64
    free-motion pass: every component within 1e-3 of its block's largest
    entry (the differentiation form's bar)."""
    prob = _free_problem()
    p32 = dataclasses.replace(prob, storage="f32")
    F, tau = np.array(prob.lat.body_force), prob.lat.tau
    J, s0, dF, dtau = AD.evaluate_free(p32, F, tau, grad=True)
    h = 1e-6
    for block in range(4):
        scale = max(np.abs(s0[:, 3 * block:3 * block + 3]).max(), 1e-12)
        for p in range(2):
            for a in range(3):
                fd = (AD.evaluate_free(_free_shift(prob, p, block, a, h), F, tau) -
                      AD.evaluate_free(_free_shift(prob, p, block, a, -h), F, tau)) / (2 * h)
                assert abs(s0[p, 3 * block + a] - fd) <= 1e-3 * scale, (block, p, a)
    e = np.array([1e-6, 0.0, 0.0])
    fd = (AD.evaluate_free(prob, F + e, tau) - AD.evaluate_free(prob, F - e, tau)) / 2e-6
    assert abs(dF[0] - fd) <= 1e-3 * abs(fd), (dF[0], fd)
    fd = (AD.evaluate_free(prob, F, tau + 1e-6) - AD.evaluate_free(prob, F, tau - 1e-6)) / 2e-6
    assert abs(dtau - fd) <= 1e-3 * abs(fd), (dtau, fd)


def _oracle_free_J(prob, F, tau):
    lat = dataclasses.replace(prob.lat, body_force=tuple(F), tau=tau)
    o = O.Oracle(lat)
    o.f[...] = prob.f0
    P = prob.ps.copy()
    dem = O.OracleDEM(P, lat)
    prm = O.DemParams(**W.dem_defaults(prob.ps, gravity=prob.gravity))
    J = 0.0
    for _ in range(prob.steps):
        o.classify(P)
        Fh, Th = o.step(P)
        J += float((prob.weights[:, :3] * Fh).sum() + (prob.weights[:, 3:] * Th).sum())
        dem.step(P, Fh, Th, prm, prob.n_sub, 1.0 / prob.n_sub)
    return J


def test_fp64_free_motion_adjoint_matches_oracle_differences():
    """The reference: central differences of the oracle's own coupled loop
    (FP64 lattice update and DEM on the CPU)."""
    prob = _free_problem(steps=12, window=5)
    F, tau = np.array(prob.lat.body_force), prob.lat.tau
    J, s0, dF, dtau = AD.evaluate_free(prob, F, tau, grad=True)
    assert abs(J - _oracle_free_J(prob, F, tau)) <= 1e-9 * abs(J)
    h = 1e-6
    for block, p, a in [(0, 0, 0), (1, 0, 2), (2, 0, 1), (3, 0, 2), (2, 1, 0), (0, 1, 1)]:
        scale = max(np.abs(s0[:, 3 * block:3 * block + 3]).max(), 1e-12)
        fd = (_oracle_free_J(_free_shift(prob, p, block, a, h), F, tau) -
              _oracle_free_J(_free_shift(prob, p, block, a, -h), F, tau)) / (2 * h)
        assert abs(s0[p, 3 * block + a] - fd) <= 5e-5 * scale, (block, p, a, s0[p, 3 * block + a], fd)


# ---------------------------------------------------------------------------
# free motion with contacts: the adjoint through the DEM's contact forces
# ---------------------------------------------------------------------------

# Centres sit off the lattice planes: a sphere of integer radius centred on
# a node has nodes exactly on its surface, whose classification flips under
# any shift, and J jumps there.

def _at_rest(lat):
    wq = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
    return np.repeat(wq[:, None], lat.ncell, axis=1)


def _pair_in_contact(steps=12, window=5):
    """Two spheres (d = 6) whose surfaces overlap by about 0.03 lu, offset
    sideways, spinning and closing at 0.06 lu/step: in contact through the
    run, with the spring-dashpot normal force and the tangential spring
    (windows of 5, so the contact state crosses two window boundaries)."""
    lat = W.LatticeSpec(32, 28, 30, (1, 0, 1), tau=0.7, body_force=(1e-5, 0.0, 0.0))
    sh = W.sphere_shape(6.0, 0.2)
    ps = W.make_particles([sh, sh], [[12.13, 14.27, 15.11], [18.08, 14.67, 15.41]],
                          [[1, 0, 0, 0]] * 2, 1.5,
                          vel=np.array([[0.03, 0.004, -0.006], [-0.03, -0.005, 0.004]]),
                          omega=np.array([[0.001, 0.002, -0.003], [0.0, -0.002, 0.001]]))
    w = np.zeros((2, 6))
    w[0, 0] = 1.0 / steps
    w[1, 1] = 0.3 / steps
    w[0, 5] = 0.2 / steps
    return AD.FreeProblem(lat=lat, ps=ps, steps=steps, window=window, storage="f64", weights=w,
                          f0=_at_rest(lat))


def _sphere_sliding_on_the_wall(steps=12, window=5):
    """A sphere (d = 8) pressed into the wall y = -1/2 by gravity (overlap
    0.03 lu) and sliding along it at 0.02 lu/step: the tangential spring
    reaches the Coulomb limit within the first step and stays there; a
    metaball above it moves freely through the fluid."""
    rng = np.random.default_rng(5)
    lat = W.LatticeSpec(32, 24, 30, (1, 0, 1), tau=0.7)
    sh = W.sphere_shape(8.0, 0.2)
    pts = np.array([[0.0, 0, 0], [1.0, 0, 0], [0.5, 0.8, 0]])
    mb = W.metaball_shape(pts, np.array([0.1, 0.12, 0.08]), 0.1, length=7.0,
                          axis=np.array([1.0, 0, 0]), samples_per_unit=4.0)
    ps = W.make_particles([sh, mb], [[14.13, 3.47, 15.21], [16.0, 14.0, 14.0]],
                          [[1, 0, 0, 0], W.random_quaternion(rng)], 2.0,
                          vel=np.array([[0.02, -0.002, 0.004], [0.01, 0.003, -0.004]]),
                          omega=np.array([[0.0, 0.001, 0.002], [0.002, 0.0, -0.001]]))
    w = np.zeros((2, 6))
    w[0, 0] = 1.0 / steps
    w[0, 1] = 0.5 / steps
    w[1, 2] = 0.4 / steps
    w[0, 3] = 0.3 / steps
    return AD.FreeProblem(lat=lat, ps=ps, steps=steps, window=window, storage="f64", weights=w,
                          f0=_at_rest(lat), gravity=(0.0, -2e-4, 0.0))


def _check_free_fd(prob, J_of, s0, rtol, comps=None):
    F, tau = np.array(prob.lat.body_force), prob.lat.tau
    h = 1e-6
    if comps is None:
        comps = [(b, p, a) for b in range(4) for p in range(prob.ps.n) for a in range(3)]
    for block, p, a in comps:
        # a sphere's rotation changes nothing: that block is zero up to the
        # differences' rounding (|J| eps / h), measured against the others
        scale = max(np.abs(s0[:, 3 * block:3 * block + 3]).max(), 1e-4 * np.abs(s0).max())
        fd = (J_of(_free_shift(prob, p, block, a, h), F, tau) -
              J_of(_free_shift(prob, p, block, a, -h), F, tau)) / (2 * h)
        got = s0[p, 3 * block + a]
        assert abs(got - fd) <= rtol * scale, (block, p, a, got, fd)


def _gpu_free_J(prob, F, tau):
    return AD.evaluate_free(prob, F, tau)


@pytest.mark.parametrize("case", ["pair", "wall"])
def test_fp64_contact_adjoint_matches_finite_differences(case):
    """Runs in contact from the first substep on: every component of
    dJ/d(x, theta, v, omega) of both initial states, and dJ/dF, dJ/dtau,
    against central differences of the same free-motion forward pass, each
    block within 2e-5 of its largest entry.  The contact moves the bodies
    (their velocities change sign or stall within the run), so a gradient
    that left the contact force out would be off by far more."""
    prob = _pair_in_contact() if case == "pair" else _sphere_sliding_on_the_wall()
    print(f"contact adjoint {case}", flush=True)
    F, tau = np.array(prob.lat.body_force), prob.lat.tau
    J, s0, dF, dtau = AD.evaluate_free(prob, F, tau, grad=True)
    assert np.isfinite(s0).all() and np.abs(s0).max() > 0
    _check_free_fd(prob, _gpu_free_J, s0, 2e-5)
    fd = (AD.evaluate_free(prob, F, tau + 1e-6) - AD.evaluate_free(prob, F, tau - 1e-6)) / 2e-6
    assert abs(dtau - fd) <= 2e-5 * abs(fd), (dtau, fd)
    e = np.array([1e-6, 0.0, 0.0])
    fd = (AD.evaluate_free(prob, F + e, tau) - AD.evaluate_free(prob, F - e, tau)) / 2e-6
    assert abs(dF[0] - fd) <= 2e-5 * max(abs(fd), np.abs(dF).max()), (dF[0], fd)


def test_fp64_contact_adjoint_matches_oracle_differences():
    """The contact pair against central differences of the oracle's own
    coupled loop (FP64 lattice update and DEM with its contact histories, on
    the CPU)."""
    prob = _pair_in_contact(steps=10, window=4)
    F, tau = np.array(prob.lat.body_force), prob.lat.tau
    J, s0, dF, dtau = AD.evaluate_free(prob, F, tau, grad=True)
    assert abs(J - _oracle_free_J(prob, F, tau)) <= 1e-9 * abs(J)
    _check_free_fd(prob, _oracle_free_J, s0, 5e-5,
                   comps=[(0, 0, 0), (0, 1, 1), (1, 0, 2), (2, 0, 0), (2, 1, 2), (3, 1, 1)])


def _chain(n):
    """n spheres (d = 4) in a row along x, neighbours overlapping by 0.01
    lu, alternately moving in +y and -y: every neighbour pair is a
    broad-phase candidate, so the contact cluster of each is the whole row."""
    lat = W.LatticeSpec(48, 16, 16, (1, 0, 1), tau=0.7)
    sh = W.sphere_shape(4.0, 0.2)
    pos = [[6.17 + 3.99 * i, 8.23, 7.91] for i in range(n)]
    vel = np.array([[0.0, 0.004 * (-1) ** i, 0.0] for i in range(n)])
    ps = W.make_particles([sh] * n, pos, [[1, 0, 0, 0]] * n, 1.5, vel=vel)
    w = np.zeros((n, 6))
    w[:, 1] = 1.0 / 6
    return AD.FreeProblem(lat=lat, ps=ps, steps=6, window=3, storage="f64", weights=w,
                          f0=_at_rest(lat))


def test_contact_adjoint_at_the_largest_cluster_and_beyond():
    """A row of 8 spheres (the largest contact cluster the adjoint
    simulates) is differentiated (three components against central
    differences); a row of 9 is refused with ESTATE naming the cluster
    rather than a gradient that leaves a particle of the cluster out."""
    prob = _chain(8)
    F, tau = np.array(prob.lat.body_force), prob.lat.tau
    J, s0, dF, dtau = AD.evaluate_free(prob, F, tau, grad=True)
    assert np.isfinite(s0).all() and np.abs(s0).max() > 0
    _check_free_fd(prob, _gpu_free_J, s0, 2e-5, comps=[(0, 0, 0), (2, 3, 1), (0, 7, 0)])
    prob = _chain(9)
    with pytest.raises(B.LbmError) as e:
        AD.evaluate_free(prob, F, tau, grad=True)
    assert e.value.code == B.LBM_ESTATE
    assert "cluster" in str(e.value)


def test_two_context_backward_matches_one_context():
    """The backward pass that replays each window on a second context beside
    the adjoint of the window after it (the forward pass's geometry kept)
    gives the gradient of the one-context pass (each replay classifying
    again), for prescribed and for free motion, over several windows."""
    prob = _problem("f64", steps=30, window=7)
    v, F, tau = prob.ps.vel.copy(), np.array(prob.lat.body_force), prob.lat.tau
    a = AD.evaluate(prob, v, F, tau, grad=True)
    b = AD.evaluate(dataclasses.replace(prob, keep_geometry=False), v, F, tau, grad=True)
    assert abs(a[0] - b[0]) <= 1e-13 * abs(b[0])
    np.testing.assert_allclose(a[1], b[1], rtol=1e-10, atol=1e-12 * np.abs(b[1]).max())
    np.testing.assert_allclose(a[2], b[2], rtol=1e-10)
    assert abs(a[3] - b[3]) <= 1e-7 * abs(b[3])
    fp = _free_problem(steps=20, window=6)
    F, tau = np.array(fp.lat.body_force), fp.lat.tau
    a = AD.evaluate_free(fp, F, tau, grad=True)
    b = AD.evaluate_free(dataclasses.replace(fp, keep_geometry=False), F, tau, grad=True)
    assert abs(a[0] - b[0]) <= 1e-13 * abs(b[0])
    for k in range(4):
        blk = slice(3 * k, 3 * k + 3)
        np.testing.assert_allclose(a[1][:, blk], b[1][:, blk], rtol=1e-9,
                                   atol=1e-11 * np.abs(b[1][:, blk]).max())
    np.testing.assert_allclose(a[2], b[2], rtol=1e-9)
    assert abs(a[3] - b[3]) <= 1e-7 * abs(b[3])
