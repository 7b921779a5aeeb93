"""Parity at the full sizes of the five workloads, in the launch
configuration the benchmark times.

c1 (40x40x80, FP64), c2 (128x128x256, FP32) and c3 (256^3, 200 bodies, FP32
and FP16) are compared with the full FP64 oracle over a few steps of a
prescribed rigid trajectory: geometry bit-exact every step, forces, torques and
populations within the storage's tolerance.  c4 (512^3, 1000 bodies, FP32) is
too large for the oracle's FP64 populations, so its geometry (owner plane,
every link record, the refill set) is compared bit-exactly on the whole
lattice, and forces and populations are compared for sampled bodies: the
oracle runs a sub-box around each sampled body holding every body that reaches
into it, with margins wider than the distance information travels in the
steps compared (two nodes per step: one by streaming, one through x_ff).
DEM is compared on all c4 bodies."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2206_11634_amd import binding as B
from paper_2206_11634_amd import workloads as W
import oracle_windows as OW
from test_gpu_parity import FORCE_TOL, POP_TOL, _compare_geometry, _run

pytestmark = pytest.mark.gpu


def _moving(ps, seed, speed, spin):
    rng = np.random.default_rng(seed)
    ps = ps.copy()
    ps.vel = rng.normal(size=(ps.n, 3)) * speed
    ps.omega = rng.normal(size=(ps.n, 3)) * spin
    return ps


def test_c1_full_size_fp64():
    lat, ps, meta = W.config_c1()
    ps = _moving(ps, 11, 0.02, 0.003)
    r = _run(lat, ps, "f64", 30, tag="c1")
    assert r["pop_err"] <= POP_TOL["f64"] and r["F"] <= FORCE_TOL["f64"] and r["T"] <= FORCE_TOL["f64"], r


def test_c2_full_size_fp32():
    lat, ps, meta = W.config_c2()
    ps = _moving(ps, 12, 0.03, 0.002)
    r = _run(lat, ps, "f32", 8, tag="c2")
    assert r["pop_err"] <= POP_TOL["f32"] and r["F"] <= FORCE_TOL["f32"] and r["T"] <= FORCE_TOL["f32"], r


@pytest.mark.parametrize("storage,classify,lattice", [("f32", "auto", 19), ("f16", "sweep", 19),
                                                      ("f32", "auto", 15)])
def test_c3_full_size(storage, classify, lattice):
    lat, ps, meta = W.config_c3()
    ps = _moving(ps, 13, 0.02, 0.002)
    r = _run(lat, ps, storage, 3, tag=f"c3 {storage} {classify} q{lattice}", classify=classify,
             lattice=lattice)
    assert r["refilled"] > 0
    assert r["pop_err"] <= POP_TOL[storage], r
    assert r["F"] <= FORCE_TOL[storage] and r["T"] <= FORCE_TOL[storage], r


# ---------------------------------------------------------------------------
# c4: whole-lattice geometry, sampled bodies for forces and populations
# ---------------------------------------------------------------------------
K_STEPS = 3


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_c4_full_size_geometry_and_sampled_bodies(storage):
    """The timed workload as the benchmark runs it: its treatment bits (1+2+8),
    both deviation storages, and its launch configuration (lbm_step_dem: the
    stream-collide pass on its masked stream beside the DEM call; the DEM's
    update of the particles is overwritten by the prescribed state of the
    next step).  The whole-lattice geometry does not depend on the storage
    and is compared in the FP32 run."""
    lat, ps, meta = W.config_c4()
    treat = meta["treatments"]
    prm = B.DemParams.make(**W.dem_defaults(ps, gravity=meta["gravity"]))
    n_sub = meta["n_sub"]
    ps = _moving(ps, 14, 0.02, 0.001)
    margin = 2 * K_STEPS + 4
    half_extra = 2 + margin
    sample = OW.sample_bodies(lat, ps, half_extra)
    traj = [W.prescribed_state(ps, lat, float(t)) for t in range(K_STEPS + 1)]

    gpu = B.Lattice.for_particles(lat, ps, storage=storage, treatments=treat)
    parts = B.DeviceParticles(ps)
    geo = O.Oracle(lat, treat=treat, fields=False) if storage == "f32" else None
    Fg, Tg = [], []
    for t in range(K_STEPS):
        parts.set_state(traj[t])
        counts = gpu.classify(parts)
        if geo is not None and t < 2:
            geo.classify(traj[t])
            _compare_geometry(gpu, geo, f"c4 step {t}")
            if t == 1:
                assert len(geo.refill_nodes) > 0
        gpu.step_dem(parts, n_sub, 1.0 / n_sub, prm)
        F, T = gpu.forces()
        Fg.append(F.cpu().numpy()[sample].copy())
        Tg.append(T.cpu().numpy()[sample].copy())
    assert counts.n_links > 2e7
    del geo
    Fg, Tg = np.array(Fg), np.array(Tg)

    for si, p in enumerate(sample):
        Fo, To, ora, lo, wdims, real = OW.run_window(lat, ps, traj, p, K_STEPS, half_extra,
                                                     treat=treat)
        eF = np.abs(Fg[:, si] - Fo).max() / np.abs(Fo).max()
        eT = np.abs(Tg[:, si] - To).max() / np.abs(To).max()
        assert eF <= FORCE_TOL[storage] and eT <= FORCE_TOL[storage], (p, eF, eT)
        # populations in the core of the sub-box, away from its artificial faces
        lnode, gnode = OW.core_fluid_nodes(lat, ora, lo, wdims, real, 2 * K_STEPS + 2)
        pick = np.random.default_rng(p).choice(len(gnode), size=min(20000, len(gnode)),
                                               replace=False)
        fg = gpu.populations(gnode[pick])
        err = np.abs(fg - ora.f[:, lnode[pick]]).max()
        assert err <= POP_TOL[storage], (p, err)
    gpu.close()


def test_c4_dem_full_size():
    """All 1000 bodies: gravity, seeded velocities, contacts wherever the
    seeded layout brings bodies together; no fluid loads (no lattice step has
    run, so F^h = T^h = 0 on both sides)."""
    lat, ps, meta = W.config_c4()
    ps = _moving(ps, 15, 0.02, 0.002)
    kw = W.dem_defaults(ps, gravity=meta["gravity"])
    n_sub, dt = meta["n_sub"], 1.0 / meta["n_sub"]
    gpu = B.Lattice.for_particles(lat, ps, storage="f32")
    parts = B.DeviceParticles(ps)
    dem = O.OracleDEM(ps, lat)
    P = ps.copy()
    zero = np.zeros((ps.n, 3))
    for _ in range(20):
        gpu.dem(parts, n_sub, dt, B.DemParams.make(**kw))
        dem.step(P, zero, zero, O.DemParams(**kw), n_sub, dt)
    G = parts.to_host(ps)
    gpu.close()
    for k in ("pos", "vel", "omega", "quat", "world_pts"):
        a, b = getattr(G, k), getattr(P, k)
        assert np.abs(a - b).max() <= 1e-9 * max(1.0, np.abs(b).max()), k


@pytest.mark.parametrize("periodic", [(1, 1, 0), (0, 0, 0)], ids=["xy_periodic", "walls"])
def test_dem_cell_grid_dense_spheres(periodic):
    """2548 spheres (d = 5.2) on a jittered 5-unit lattice filling a 70^3 box,
    periodic in x and y or walled on every side: every body presses on its
    neighbours (across the periodic faces too), so the broad phase on the
    cell grid (taken from 2048 particles on) must find the same pairs as the
    oracle's all-pairs test."""
    rng = np.random.default_rng(21)
    lat = W.LatticeSpec(70, 70, 70, periodic, tau=0.6)
    sh = W.sphere_shape(5.2, 0.1)
    g = (np.arange(14) + 0.5) * 5.0
    z = 4.0 + 5.0 * np.arange(13)
    X, Y, Z = np.meshgrid(g, g, z, indexing="ij")
    pos = np.stack([X.ravel(), Y.ravel(), Z.ravel()], -1) + rng.normal(size=(14 * 14 * 13, 3)) * 0.15
    n = len(pos)
    quats = np.array([W.random_quaternion(rng) for _ in range(n)])
    ps = W.make_particles([sh] * n, pos, quats, 1.5)
    ps = _moving(ps, 22, 0.02, 0.002)
    kw = W.dem_defaults(ps, gravity=(0.0, 0.0, -1e-4))
    gpu = B.Lattice.for_particles(lat, ps, storage="f32")
    parts = B.DeviceParticles(ps)
    dem = O.OracleDEM(ps, lat)
    P = ps.copy()
    zero = np.zeros((n, 3))
    for _ in range(8):
        gpu.dem(parts, 10, 0.1, B.DemParams.make(**kw))
        dem.step(P, zero, zero, O.DemParams(**kw), 10, 0.1)
    G = parts.to_host(ps)
    gpu.close()
    assert np.abs(P.pos - ps.pos).max() > 1e-3  # the contacts moved the bodies
    for k in ("pos", "vel", "omega", "quat", "world_pts"):
        a, b = getattr(G, k), getattr(P, k)
        assert np.abs(a - b).max() <= 1e-9 * max(1.0, np.abs(b).max()), k


def test_dem_cell_grid_thin_periodic_axis():
    """2048 spheres in two sheets on a periodic axis only 15 nodes long, so the
    grid has two cells along it and both neighbours of a cell are the same
    cell (visited once, or every pair across it would be listed twice);
    contacts across the sheets and across the periodic y faces."""
    rng = np.random.default_rng(31)
    sh = W.sphere_shape(5.2, 0.1)
    y = (np.arange(32) + 0.5) * 5.0
    z = 4.0 + 5.0 * np.arange(32)
    Y, Z = np.meshgrid(y, z, indexing="ij")
    pos = np.concatenate([np.stack([np.full(Y.size, x0), Y.ravel(), Z.ravel()], -1)
                          for x0 in (3.0, 8.0)])
    pos = pos + rng.normal(size=pos.shape) * 0.15
    n = len(pos)
    ps = W.make_particles([sh] * n, pos, np.array([W.random_quaternion(rng) for _ in range(n)]),
                          1.5)
    ps = _moving(ps, 32, 0.02, 0.002)
    lat = W.LatticeSpec(15, 160, 167, (1, 1, 0), tau=0.6)
    kw = W.dem_defaults(ps, gravity=(0.0, 0.0, -1e-4))
    gpu = B.Lattice.for_particles(lat, ps, storage="f32")
    parts = B.DeviceParticles(ps)
    dem = O.OracleDEM(ps, lat)
    P = ps.copy()
    zero = np.zeros((n, 3))
    for _ in range(6):
        gpu.dem(parts, 10, 0.1, B.DemParams.make(**kw))
        dem.step(P, zero, zero, O.DemParams(**kw), 10, 0.1)
    G = parts.to_host(ps)
    gpu.close()
    assert np.abs(P.pos - ps.pos).max() > 1e-3
    for k in ("pos", "vel", "omega", "quat", "world_pts"):
        a, b = getattr(G, k), getattr(P, k)
        assert np.abs(a - b).max() <= 1e-9 * max(1.0, np.abs(b).max()), k


# ---------------------------------------------------------------------------
# long replay runs against the oracle's stored series
# (tests/golden/make_drag_reference.py writes them with the oracle alone)
# ---------------------------------------------------------------------------

def _stored_reference(name):
    from pathlib import Path
    lat, ps, steps, treat, desc = W.drag_case(name)
    path = Path(__file__).resolve().parent / "golden" / f"drag_{name}.npz"
    ref = np.load(path, allow_pickle=False)
    assert str(ref["fingerprint"]) == W.fingerprint(lat, ps, steps, treat), \
        "stored oracle series made from other inputs: run tests/golden/make_drag_reference.py"
    return lat, ps, steps, treat, ref


def _replay_forces(lat, ps, steps, treat, storage):
    import torch
    traj = B.DeviceTrajectory([W.prescribed_state(ps, lat, float(n)) for n in range(steps + 1)])
    gpu = B.Lattice.for_particles(lat, ps, storage=storage, treatments=treat)
    out = torch.zeros((steps, ps.n, 6), dtype=torch.float64, device=gpu.device)
    for k in range(steps):
        gpu.classify(traj[k])
        gpu.step(traj[k])
        f, t = gpu.forces()
        out[k, :, :3] = f
        out[k, :, 3:] = t
    res = out.cpu().numpy()
    gpu.close()
    return res


def _series_error(g, ref):
    """Per body: max over steps |X_gpu - X_oracle| / max over steps |X_oracle|."""
    e = []
    for sl, R in ((slice(0, 3), ref["F"]), (slice(3, 6), ref["T"])):
        num = np.linalg.norm(g[:, :, sl] - R, axis=2).max(0)
        den = np.linalg.norm(R, axis=2).max(0)
        e.append(num / den)
    return np.max(e, axis=0)


@pytest.mark.parametrize("name,storage", [("c2", "f32"), ("c3", "f32"), ("c3", "f16")])
def test_drag_series_against_the_oracle(name, storage):
    """c2: the 24 lu metaball descending and tumbling for 2000 steps; c3: the
    200-body suspension for 100 steps.  Force and torque of every body at
    every step within the storage's drag bar of the FP64 oracle."""
    lat, ps, steps, treat, ref = _stored_reference(name)
    g = _replay_forces(lat, ps, steps, treat, storage)
    err = _series_error(g, ref)
    assert err.max() <= FORCE_TOL[storage], (name, storage, err.max(), int(err.argmax()))
