"""Parity of the HIP path (through the C-ABI) with the FP64 oracle.

Geometry (owners, link records including q, refill sets) must be bit-exact.
Populations and forces must agree within the storage's tolerance:
  FP64 plain: populations 1e-12, force/torque relative 1e-10;
  FP32 deviations: populations 2e-7, force/torque relative 1e-4;
  FP16 deviations: populations 1e-4, force/torque relative 2e-2.
Relative force error = max over steps of |F_gpu - F_oracle| divided by the
largest |F_oracle| of that particle over the run.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2206_11634_amd import binding as B
from paper_2206_11634_amd import workloads as W

pytestmark = pytest.mark.gpu

POP_TOL = {"f64": 1e-12, "f32": 2e-7, "f16": 1e-4}
FORCE_TOL = {"f64": 1e-10, "f32": 1e-4, "f16": 2e-2}


def _compare_geometry(gpu, ora, tag):
    own = gpu.owner()
    assert np.array_equal(own, ora.owner), f"{tag}: owner planes differ"
    L = gpu.links()
    R = ora.links
    assert len(L["node"]) == len(R), f"{tag}: link count {len(L['node'])} vs {len(R)}"
    assert np.array_equal(L["node"], R.node), tag
    assert np.array_equal(L["d"], R.d), tag
    assert np.array_equal(L["kind"], R.kind), tag
    assert np.array_equal(L["part"], R.part), tag
    assert np.array_equal(L["q"].view(np.uint64), R.q.view(np.uint64)), f"{tag}: q not bit-exact"
    # no two reconstructing links write the same ghost slot (node, d-bar)
    w = L["kind"] != B.LINK_MISSING
    key = L["node"][w].astype(np.int64) * 32 + L["d"][w]
    assert np.unique(key).size == key.size, f"{tag}: two links write one ghost slot"
    nodes, parts = gpu.refill()
    assert np.array_equal(nodes, ora.refill_nodes), f"{tag}: refill sets differ"
    if len(nodes):
        assert np.array_equal(parts, ora.owner_prev[nodes] - 1)


def _run(lat, ps, storage, steps, treat=3, check_geometry=True, tag="", classify="auto",
         lattice=19, exact_forces=False):
    gpu = B.Lattice.for_particles(lat, ps, storage=storage, treatments=treat, classify=classify,
                                  lattice=lattice, exact_forces=exact_forces)
    parts = B.DeviceParticles(ps)
    ora = O.Oracle(lat, Q=lattice, treat=treat)
    Fo_all, Fg_all, To_all, Tg_all = [], [], [], []
    refilled = 0
    for n in range(steps):
        P = W.prescribed_state(ps, lat, float(n))
        parts.set_state(P)
        gpu.classify(parts)
        ora.classify(P)
        if check_geometry:
            _compare_geometry(gpu, ora, f"{tag} step {n}")
        refilled += len(ora.refill_nodes)
        gpu.step(parts)
        Fo, To = ora.step(P)
        Fg, Tg = (t.cpu().numpy().copy() for t in gpu.forces())
        Fo_all.append(Fo), To_all.append(To), Fg_all.append(Fg), Tg_all.append(Tg)
    fg = gpu.populations()
    fl = ora.owner == 0
    pop_err = np.abs(fg[:, fl] - ora.f[:, fl]).max()
    gpu.close()
    res = dict(pop_err=pop_err, refilled=refilled)
    for name, g, o in (("F", Fg_all, Fo_all), ("T", Tg_all, To_all)):
        g, o = np.array(g), np.array(o)
        scale = np.abs(o).max(axis=(0, 2))
        err = np.abs(g - o).max(axis=(0, 2)) / np.maximum(scale, 1e-30)
        res[name] = err.max() if len(err) else 0.0
    return res


GEOM_CASES = [
    dict(seed=1, dims=(28, 20, 26), periodic=(1, 0, 1), n_particles=3),
    dict(seed=2, dims=(27, 26, 28), periodic=(1, 1, 1), n_particles=3),
    dict(seed=3, dims=(17, 21, 19), periodic=(0, 0, 0), n_particles=3),
    dict(seed=4, dims=(24, 27, 18), periodic=(0, 1, 0), n_particles=4),
]


@pytest.mark.parametrize("classify", ["balls", "sweep"])
@pytest.mark.parametrize("case", GEOM_CASES, ids=lambda c: f"seed{c['seed']}")
def test_geometry_and_plain_fp64_step_parity(case, classify):
    """Both classification schemes (owner clearing, flags and refill detection
    by per-particle ball walks, or by one lattice sweep) must give the
    oracle's geometry bit for bit."""
    lat, ps = W.tiny_case(case["seed"], dims=case["dims"], periodic=case["periodic"],
                          n_particles=case["n_particles"], diameter_range=(4.0, 7.0),
                          speed=0.06, spin=0.006, u0=(0.02, -0.01, 0.005))
    r = _run(lat, ps, "f64", 8, tag=f"seed{case['seed']} {classify}", classify=classify)
    assert r["refilled"] > 0
    assert r["pop_err"] < POP_TOL["f64"], r
    assert r["F"] < FORCE_TOL["f64"] and r["T"] < FORCE_TOL["f64"], r


TREAT_PLAIN = B.TREAT_VIBB | B.TREAT_MISSING
TREAT_TIMED = B.TREAT_VIBB | B.TREAT_MISSING | B.TREAT_NEQ_SPLIT   # the 512^3 workload's bits


@pytest.mark.parametrize("classify", ["balls", "sweep"])
@pytest.mark.parametrize("treat", [TREAT_PLAIN, TREAT_TIMED], ids=["bits3", "bits11"])
@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_deviation_storage_parity(storage, treat, classify):
    """FP32 and FP16 deviation storage against the FP64 oracle under both
    classification schemes and both treatment sets (bits 1+2, and 1+2+8 as
    the 512^3 workload runs)."""
    lat, ps = W.tiny_case(7, dims=(28, 22, 27), periodic=(1, 0, 1), n_particles=4,
                          diameter_range=(5.0, 8.0), speed=0.05, spin=0.005,
                          u0=(0.03, 0.0, 0.01), body_force=(1e-5, 0.0, 0.0))
    r = _run(lat, ps, storage, 8, treat=treat, tag=f"{storage} treat{treat} {classify}",
             classify=classify)
    assert r["pop_err"] < POP_TOL[storage], r
    assert r["F"] < FORCE_TOL[storage] and r["T"] < FORCE_TOL[storage], r


def test_ragged_multi_tile_lattice_with_walls_and_missing_points():
    """45 x 38 x 33 nodes (not a multiple of the 256-thread tile), walls in y,
    bodies close to each other and to a wall."""
    lat, ps = W.tiny_case(12, dims=(45, 38, 33), periodic=(1, 0, 1), n_particles=6,
                          diameter_range=(6.0, 10.0), speed=0.06, spin=0.006,
                          u0=(0.02, 0.0, -0.01))
    r = _run(lat, ps, "f32", 5, tag="ragged")
    assert r["pop_err"] < POP_TOL["f32"], r
    assert r["F"] < FORCE_TOL["f32"], r


@pytest.mark.parametrize("treat", [B.TREAT_VIBB, B.TREAT_MISSING, 0,
                                   B.TREAT_VIBB | B.TREAT_MISSING | B.TREAT_EXACT_Q,
                                   B.TREAT_VIBB | B.TREAT_MISSING | B.TREAT_NEQ_SPLIT])
def test_treatment_switches(treat):
    lat, ps = W.tiny_case(5, dims=(28, 26, 18), periodic=(1, 1, 0), n_particles=3,
                          diameter_range=(5.0, 7.0), speed=0.06, spin=0.006, u0=(0.01, 0.0, 0.0))
    r = _run(lat, ps, "f64", 4, treat=treat, tag=f"treat{treat}")
    assert r["pop_err"] < POP_TOL["f64"] and r["F"] < FORCE_TOL["f64"], r


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("lattice", [19, 15])
def test_poiseuille_channel_without_particles(storage, lattice):
    tau = 0.5 + np.sqrt(3.0) / 4.0
    H, g = 12, 1e-6
    lat = W.LatticeSpec(5, H, 3, (1, 0, 1), tau=tau, body_force=(g, 0, 0))
    ps = W.make_particles([], np.zeros((0, 3)), np.zeros((0, 4)), 1.0)
    gpu = B.Lattice(lat, storage=storage, lattice=lattice)
    parts = B.DeviceParticles(ps)
    ora = O.Oracle(lat, Q=lattice)
    ora.classify(ps)
    gpu.classify(parts)
    for _ in range(300):
        gpu.step(parts)
        ora.step(ps)
    fg = gpu.populations()
    assert np.abs(fg - ora.f).max() < (1e-13 if storage == "f64" else 1e-8)
    gpu.close()


def test_rest_state_is_exact_in_deviation_storage():
    """Particles and fluid at rest: the FP32 and FP16 deviations stay exactly 0."""
    lat, ps = W.tiny_case(11, dims=(28, 16, 14), periodic=(1, 0, 0), n_particles=3)
    for storage in ("f32", "f16"):
        gpu = B.Lattice.for_particles(lat, ps, storage=storage)
        parts = B.DeviceParticles(ps)
        for _ in range(5):
            gpu.classify(parts)
            gpu.step(parts)
        F, T = (t.cpu().numpy() for t in gpu.forces())
        own = gpu.owner()
        f = gpu.populations()
        w = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
        assert np.abs(f[:, own == 0] - w[:, None]).max() < 1e-16
        assert np.abs(F).max() < 1e-13 and np.abs(T).max() < 1e-12
        gpu.close()


def test_dem_parity_with_contacts():
    lat = W.LatticeSpec(48, 40, 40, (1, 0, 1))
    rng = np.random.default_rng(31)
    shapes = [W.sphere_shape(10.0, 0.3)]
    pts = np.array([[0.0, 0, 0], [1.0, 0, 0], [0.5, 0.7, 0]])
    shapes.append(W.metaball_shape(pts, rng.uniform(0.5, 1.5, 3) * 0.2, 0.3, d_eq=10.0,
                                   samples_per_unit=3.0))
    shapes.append(W.sphere_shape(8.0, 0.3))
    pos = [[14.0, 20.0, 20.0], [24.6, 20.5, 19.8], [20.0, 4.0, 21.0]]
    quats = [W.random_quaternion(rng) for _ in range(3)]
    ps = W.make_particles(shapes, pos, quats, 1.5,
                          vel=np.array([[0.02, 0, 0], [-0.02, 0.0, 0.0], [0.0, -0.02, 0.0]]),
                          omega=np.array([[0, 0, 0.01], [0.0, 0.005, 0], [0.0, 0.0, 0.0]]))
    kn = 2.0
    prm_o = O.DemParams(kn=kn, eta_n=3.0, kt=kn / 2, eta_t=0.5, mu_s=0.3,
                        gravity=(0.0, -1e-4, 0.0), rho_f=1.0)
    prm_g = B.DemParams.make(kn=kn, eta_n=3.0, kt=kn / 2, eta_t=0.5, mu_s=0.3,
                             gravity=(0.0, -1e-4, 0.0), rho_f=1.0)
    gpu = B.Lattice.for_particles(lat, ps, storage="f64")
    parts = B.DeviceParticles(ps)
    dem = O.OracleDEM(ps, lat)
    P = ps.copy()
    Fh = np.zeros((3, 3))
    for n in range(30):
        gpu.dem(parts, 10, 0.1, prm_g)
        dem.step(P, Fh, Fh, prm_o, 10, 0.1)
    G = parts.to_host(ps)
    gpu.close()
    assert np.abs(dem.fc).max() > 0 or np.abs(P.vel - ps.vel).max() > 1e-3
    for k in ("pos", "vel", "omega", "quat", "world_pts"):
        a, b = getattr(G, k), getattr(P, k)
        assert np.abs(a - b).max() <= 1e-9 * max(1.0, np.abs(b).max()), k


def test_dem_parity_sliding_and_glancing_contacts():
    """Contacts whose tangential force reaches the Coulomb limit, under
    gravity tilted 20 degrees against the floor: a sphere launched sliding
    with spin on the floor (it slides, then rolls), a flat metaball resting
    on the floor, and a sphere striking it at a glancing angle with a
    tangential velocity; the second pair runs without tangential damping,
    so the spring's reset length after the Coulomb limit sets the force.
    600 DEM calls of 10 substeps, FP64 on both sides."""
    lat = W.LatticeSpec(96, 64, 48, (1, 1, 0))
    g, th = 1e-4, np.radians(20.0)
    sh_s, sh_m = W.sphere_shape(10.0, 0.1), W.square_metaball(12.0, 0.2)
    ps = W.make_particles([sh_s, sh_m, sh_s],
                          [[20.0, 20.0, -0.5 + 5.0 - 0.01], [60.0, 30.0, 6.0],
                           [52.0, 30.3, 15.5]],
                          [[1.0, 0, 0, 0], [np.cos(0.05), np.sin(0.05), 0, 0], [1.0, 0, 0, 0]],
                          np.array([2.0, 1.5, 2.0]),
                          vel=np.array([[0.01, 0.004, 0.0], [0.0, 0.0, 0.0], [0.012, 0.003, -0.006]]),
                          omega=np.array([[0.0, 0.0, 0.002], [0.0, 0.0, 0.0], [0.004, 0.0, -0.003]]))
    m = ps.mass.min()
    kn = (ps.mass[0] - ps.volume[0]) * g / 0.01
    kw = dict(kn=kn, eta_n=1.4 * np.sqrt(m * kn), kt=kn / 2, eta_t=0.0, mu_s=0.3,
              gravity=(g * np.sin(th), 0.0, -g * np.cos(th)), rho_f=1.0)
    gpu = B.Lattice.for_particles(lat, ps, storage="f64")
    parts = B.DeviceParticles(ps)
    dem = O.OracleDEM(ps, lat)
    P = ps.copy()
    Fh = np.zeros((3, 3))
    slid = rolled = False
    for n in range(600):
        gpu.dem(parts, 10, 0.1, B.DemParams.make(**kw))
        dem.step(P, Fh, Fh, O.DemParams(**kw), 10, 0.1)
        slip = P.vel[0, 0] - P.omega[0, 1] * 5.0
        slid |= slip > 0.2 * P.vel[0, 0]
        rolled |= slid and abs(slip) < 0.02 * abs(P.vel[0, 0])
    G = parts.to_host(ps)
    gpu.close()
    assert slid and rolled
    assert np.abs(P.vel[2] - ps.vel[2]).max() > 1e-3   # the glancing pair touched
    for k in ("pos", "vel", "omega", "quat", "world_pts"):
        a, b = getattr(G, k), getattr(P, k)
        assert np.abs(a - b).max() <= 1e-9 * max(1.0, np.abs(b).max()), k


@pytest.mark.parametrize("ang", [0.0, 0.6])
def test_dem_parity_tilted_flat_pair(ang):
    """Flat square metaballs meeting face to face and at an angle (the
    stationary point of M_A + M_B enters one internal body before contact):
    1500 DEM steps through approach, contact and rebound."""
    lat = W.LatticeSpec(150, 150, 250, (0, 0, 0))
    sh = W.square_metaball()
    ps = W.make_particles([sh, sh], [[75.0, 75.0, 120.0], [79.0, 75.0, 104.5]],
                          [[1.0, 0, 0, 0], [np.cos(ang / 2), 0, np.sin(ang / 2), 0]], 1.3,
                          vel=np.array([[0, 0, -0.005], [0, 0, 0]]))
    kw = W.dem_defaults(ps)
    gpu = B.Lattice.for_particles(lat, ps, storage="f64")
    parts = B.DeviceParticles(ps)
    dem = O.OracleDEM(ps, lat)
    P = ps.copy()
    Fh = np.zeros((2, 3))
    touched = False
    for n in range(1500):
        gpu.dem(parts, 10, 0.1, B.DemParams.make(**kw))
        dem.step(P, Fh, Fh, O.DemParams(**kw), 10, 0.1)
        touched |= bool(np.abs(dem.fc).max() > 0)
    G = parts.to_host(ps)
    gpu.close()
    assert touched
    for k in ("pos", "vel", "omega", "quat"):
        a, b = getattr(G, k), getattr(P, k)
        assert np.abs(a - b).max() <= 1e-9 * max(1.0, np.abs(b).max()), k


# ---------------------------------------------------------------------------
# D3Q15, the paper's lattice (Sec. 2.2): the same kernels built for 15
# directions, against the oracle's D3Q15 stencil
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("classify", ["balls", "sweep"])
@pytest.mark.parametrize("case", GEOM_CASES[:3], ids=lambda c: f"seed{c['seed']}")
def test_d3q15_geometry_and_plain_fp64_step_parity(case, classify):
    lat, ps = W.tiny_case(case["seed"], dims=case["dims"], periodic=case["periodic"],
                          n_particles=case["n_particles"], diameter_range=(4.0, 7.0),
                          speed=0.06, spin=0.006, u0=(0.02, -0.01, 0.005))
    r = _run(lat, ps, "f64", 8, tag=f"q15 seed{case['seed']} {classify}", classify=classify,
             lattice=15)
    assert r["refilled"] > 0
    assert r["pop_err"] < POP_TOL["f64"], r
    assert r["F"] < FORCE_TOL["f64"] and r["T"] < FORCE_TOL["f64"], r


@pytest.mark.parametrize("treat", [TREAT_PLAIN, TREAT_TIMED], ids=["bits3", "bits11"])
@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_d3q15_deviation_storage_parity(storage, treat):
    lat, ps = W.tiny_case(7, dims=(28, 22, 27), periodic=(1, 0, 1), n_particles=4,
                          diameter_range=(5.0, 8.0), speed=0.05, spin=0.005,
                          u0=(0.03, 0.0, 0.01), body_force=(1e-5, 0.0, 0.0))
    r = _run(lat, ps, storage, 8, treat=treat, tag=f"q15 {storage} treat{treat}", lattice=15)
    assert r["pop_err"] < POP_TOL[storage], r
    assert r["F"] < FORCE_TOL[storage] and r["T"] < FORCE_TOL[storage], r


@pytest.mark.parametrize("treat", [B.TREAT_VIBB | B.TREAT_MISSING | B.TREAT_EXACT_Q,
                                   B.TREAT_MISSING, B.TREAT_VIBB | B.TREAT_MISSING | B.TREAT_NEQ_SPLIT])
def test_d3q15_treatment_switches(treat):
    lat, ps = W.tiny_case(5, dims=(28, 26, 18), periodic=(1, 1, 0), n_particles=3,
                          diameter_range=(5.0, 7.0), speed=0.06, spin=0.006, u0=(0.01, 0.0, 0.0))
    r = _run(lat, ps, "f64", 4, treat=treat, tag=f"q15 treat{treat}", lattice=15)
    assert r["pop_err"] < POP_TOL["f64"] and r["F"] < FORCE_TOL["f64"], r


def test_classify_rejects_bad_particles_and_keeps_the_geometry():
    """A particle state that fails the boxes' check (a centre outside [0, n)
    on a periodic axis) is reported as EINVAL by lbm_classify_nodes, whose
    kernels then leave the owner planes, flags and lists alone; a valid
    classification afterwards gives the oracle's geometry."""
    lat, ps = W.tiny_case(1, dims=(28, 20, 26), periodic=(1, 0, 1), n_particles=3,
                          diameter_range=(4.0, 7.0), speed=0.06, spin=0.006)
    gpu = B.Lattice.for_particles(lat, ps, storage="f64")
    parts = B.DeviceParticles(ps)
    gpu.classify(parts)
    own0 = gpu.owner()
    bad = ps.copy()
    bad.pos[0, 0] = -5.0
    bad.refresh_world()
    parts.set_state(bad)
    with pytest.raises(B.LbmError) as e:
        gpu.classify(parts)
    assert e.value.code == B.LBM_EINVAL
    assert np.array_equal(gpu.owner(), own0)
    P1 = W.prescribed_state(ps, lat, 1.0)
    parts.set_state(P1)
    gpu.classify(parts)
    ora = O.Oracle(lat, fields=False)
    ora.classify(ps)
    ora.classify(P1)
    _compare_geometry(gpu, ora, "after a rejected state")
    gpu.close()


def test_async_classification_matches_the_synchronous_one():
    """lbm_classify_nodes_async builds the same owners, links and refills as
    lbm_classify_nodes (the step then covers the whole link capacity): over a
    moving run the populations agree bit for bit and the forces to rounding;
    the link list is not readable until a synchronous classification."""
    lat, ps = W.tiny_case(3, dims=(30, 22, 26), periodic=(1, 0, 1), n_particles=3,
                          diameter_range=(4.0, 7.0), speed=0.08, spin=0.01)
    runs = []
    for sync in (True, False):
        gpu = B.Lattice.for_particles(lat, ps, storage="f32")
        parts = B.DeviceParticles(ps)
        gpu.classify(parts)
        forces = []
        for k in range(14):
            gpu.step(parts)
            F, T = gpu.forces()
            forces.append(np.concatenate([F.cpu().numpy(), T.cpu().numpy()], axis=1))
            parts.set_state(W.prescribed_state(ps, lat, float(k + 1)))
            gpu.classify(parts, sync=sync)
        if not sync:
            with pytest.raises(B.LbmError) as e:
                gpu.links()
            assert e.value.code == B.LBM_ESTATE
        gpu.sync()
        runs.append((gpu.populations(), gpu.owner(), np.array(forces)))
        gpu.close()
    (fa, oa, Fa), (fb, ob, Fb) = runs
    np.testing.assert_array_equal(fa, fb)
    np.testing.assert_array_equal(oa, ob)
    np.testing.assert_allclose(Fb, Fa, rtol=1e-12, atol=1e-15 * np.abs(Fa).max())


def test_async_classification_latches_a_rejected_particle():
    """A state that fails the boxes' check under the asynchronous call is
    reported by the next lbm_synchronize as EINVAL, and the context is failed
    (the steps in between ran on geometry that was not rebuilt)."""
    lat, ps = W.tiny_case(1, dims=(28, 20, 26), periodic=(1, 0, 1), n_particles=3,
                          diameter_range=(4.0, 7.0), speed=0.06, spin=0.006)
    gpu = B.Lattice.for_particles(lat, ps, storage="f32")
    parts = B.DeviceParticles(ps)
    gpu.classify(parts)
    gpu.step(parts)
    bad = ps.copy()
    bad.pos[0, 0] = -5.0
    bad.refresh_world()
    parts.set_state(bad)
    gpu.classify(parts, sync=False)
    with pytest.raises(B.LbmError) as e:
        gpu.sync()
    assert e.value.code == B.LBM_EINVAL
    with pytest.raises(B.LbmError) as e:
        gpu.step(parts)
    assert e.value.code == B.LBM_ESTATE
    gpu.close()


def test_non_finite_forces_are_reported_and_fail_the_context():
    """A population set to NaN next to a body (forced from the host) makes the
    step's momentum-exchange sums non-finite; the next classification reports
    ENUMERIC and every later call ESTATE."""
    lat, ps = W.tiny_case(2, dims=(27, 26, 28), periodic=(1, 1, 1), n_particles=3,
                          diameter_range=(4.0, 7.0))
    gpu = B.Lattice.for_particles(lat, ps, storage="f32")
    parts = B.DeviceParticles(ps)
    gpu.classify(parts)
    gpu.step(parts)
    gpu.classify(parts)
    L = gpu.links()
    f = gpu.populations()
    d, node = int(L["d"][0]), int(L["node"][0])
    e = np.array(O.stencil(19)[0][d])
    x = np.array([node % lat.nx, (node // lat.nx) % lat.ny, node // (lat.nx * lat.ny)]) - e
    x %= np.array(lat.dims)
    f[d, x[0] + lat.nx * (x[1] + lat.ny * x[2])] = np.nan
    gpu.set_populations(f)
    gpu.step(parts)
    with pytest.raises(B.LbmError) as err:
        gpu.classify(parts)
    assert err.value.code == B.LBM_ENUMERIC
    with pytest.raises(B.LbmError) as err:
        gpu.step(parts)
    assert err.value.code == B.LBM_ESTATE
    gpu.close()


@pytest.mark.parametrize("storage,lattice", [("f64", 19), ("f32", 19), ("f16", 19), ("f64", 15)])
def test_moments_export_matches_oracle(storage, lattice):
    """lbm_get_moments: rho and u = (sum f e + F/2)/rho of every fluid node
    against the oracle's moments of its populations, after moving steps with
    refills and a body force."""
    lat, ps = W.tiny_case(7, dims=(28, 22, 27), periodic=(1, 0, 1), n_particles=4,
                          diameter_range=(5.0, 8.0), speed=0.05, spin=0.005,
                          u0=(0.03, 0.0, 0.01), body_force=(1e-5, 0.0, 0.0))
    gpu = B.Lattice.for_particles(lat, ps, storage=storage, lattice=lattice)
    parts = B.DeviceParticles(ps)
    ora = O.Oracle(lat, Q=lattice)
    for n in range(6):
        P = W.prescribed_state(ps, lat, float(n))
        parts.set_state(P)
        gpu.classify(parts)
        ora.classify(P)
        gpu.step(parts)
        ora.step(P)
    rho_g, u_g = gpu.moments()
    rho_o, u_o = ora.moments()
    fl = ora.owner == 0
    tol = {"f64": 1e-13, "f32": 1e-6, "f16": 2e-4}[storage]
    assert np.abs(rho_g[fl] - rho_o[fl]).max() < tol
    assert np.abs(u_g[fl] - u_o[fl]).max() < tol
    gpu.close()


@pytest.mark.parametrize("dims", [(28, 22, 27), (27, 22, 26)], ids=["even_nx", "odd_nx"])
def test_fp16_pair_and_single_node_bulk_paths(dims):
    """FP16 storage runs the bulk pass two nodes per thread when nx is even
    and one node per thread otherwise; both against the oracle, with walls on
    y and z so that pairs pull through walls too."""
    lat, ps = W.tiny_case(9, dims=dims, periodic=(1, 0, 0), n_particles=3,
                          diameter_range=(5.0, 7.0), speed=0.05, spin=0.005,
                          u0=(0.02, 0.01, 0.0), body_force=(1e-5, 0.0, 0.0))
    r = _run(lat, ps, "f16", 8, tag=f"f16 {dims}")
    assert r["pop_err"] < POP_TOL["f16"], r
    assert r["F"] < FORCE_TOL["f16"] and r["T"] < FORCE_TOL["f16"], r


# ---------------------------------------------------------------------------
# limits: a body larger than the FP32 estimate covers, the most control points
# a body may have, one more than that
# ---------------------------------------------------------------------------

def test_large_body_geometry_takes_the_fp64_path():
    """A sphere of radius 130 (node box half-width 133 > 127, where the
    classification's FP32 estimate is not trusted and every node takes the
    FP64 sum) in a 272^3 periodic box: owners, links and q bit-exact."""
    lat = W.LatticeSpec(272, 272, 272, (1, 1, 1), tau=0.7)
    ps = W.make_particles([W.sphere_shape(260.0, 0.1)], [[136.3, 135.8, 136.1]],
                          [[1.0, 0, 0, 0]], 1.5, vel=[[0.01, 0.0, 0.0]])
    assert ps.box_half() > 127
    gpu = B.Lattice.for_particles(lat, ps, storage="f32")
    parts = B.DeviceParticles(ps)
    ora = O.Oracle(lat, fields=False)
    for n in range(2):
        P = W.prescribed_state(ps, lat, float(n))
        parts.set_state(P)
        gpu.classify(parts)
        ora.classify(P)
        _compare_geometry(gpu, ora, f"r130 step {n}")
    gpu.close()


def _cluster_shape(rng, n_pts, length):
    pts = rng.normal(size=(n_pts, 3)) * 0.6
    return W.metaball_shape(pts, rng.uniform(0.5, 1.5, n_pts) * 0.05, 0.1, length=length,
                            axis=np.array([1.0, 0.0, 0.0]), samples_per_unit=1.0)


def test_sixty_four_control_points_parity():
    rng = np.random.default_rng(64)
    sh = _cluster_shape(rng, 64, 10.0)
    lat = W.LatticeSpec(30, 28, 26, (1, 0, 1), tau=0.7, u0=(0.02, 0.0, 0.0))
    ps = W.make_particles([sh], [[15.2, 13.9, 13.1]], [W.random_quaternion(rng)], 1.5,
                          vel=[[0.03, 0.01, 0.0]], omega=[[0.0, 0.01, 0.005]])
    r = _run(lat, ps, "f64", 5, tag="64 points")
    assert r["pop_err"] < POP_TOL["f64"] and r["F"] < FORCE_TOL["f64"], r


def test_more_than_sixty_four_control_points_is_rejected():
    rng = np.random.default_rng(65)
    sh = _cluster_shape(rng, 65, 10.0)
    lat = W.LatticeSpec(40, 40, 40, (0, 0, 0), tau=0.7)
    ps = W.make_particles([sh], [[20.2, 19.9, 20.1]], [[1.0, 0, 0, 0]], 1.5)
    gpu = B.Lattice.for_particles(lat, ps, storage="f32")
    parts = B.DeviceParticles(ps)
    with pytest.raises(B.LbmError) as e:
        gpu.classify(parts)
    assert e.value.code == B.LBM_EINVAL
    assert b"more than 64" in B.load().lbm_last_error(gpu.ctx)
    gpu.close()


def test_dem_more_candidate_partners_than_history_records_is_reported():
    """A sphere ringed by 40 small spheres within the broad phase's reach
    (centres 4.2 lu apart, reach 2.9 + 0.9 + R_s + 1/2): particle 0 has 40
    candidate partners of higher index, more than its 32 history records.
    dem_step leaves the extra pairs out and latches it; lbm_synchronize
    reports ECAPACITY and the context is failed."""
    lat = W.LatticeSpec(40, 40, 40, (1, 1, 1))
    k = np.arange(40) + 0.5
    th, ph = np.arccos(1 - 2 * k / 40), np.pi * (1 + 5 ** 0.5) * k
    ring = 4.2 * np.stack([np.cos(ph) * np.sin(th), np.sin(ph) * np.sin(th), np.cos(th)], 1)
    c = np.array([20.0, 20.0, 20.0])
    shapes = [W.sphere_shape(6.0, 0.1)] + [W.sphere_shape(2.0, 0.1)] * 40
    ps = W.make_particles(shapes, np.vstack([c, c + ring]), [[1.0, 0, 0, 0]] * 41, 1.5)
    gpu = B.Lattice.for_particles(lat, ps, storage="f64")
    parts = B.DeviceParticles(ps)
    gpu.dem(parts, 2, 0.1, B.DemParams.make(**W.dem_defaults(ps)))
    with pytest.raises(B.LbmError) as e:
        gpu.sync()
    assert e.value.code == B.LBM_ECAPACITY
    assert "candidate contact partners" in str(e.value)
    with pytest.raises(B.LbmError) as e:
        gpu.dem(parts, 2, 0.1, B.DemParams.make(**W.dem_defaults(ps)))
    assert e.value.code == B.LBM_ESTATE
    gpu.close()


@pytest.mark.parametrize("storage,lattice", [("f64", 19), ("f32", 19), ("f16", 19), ("f32", 15)])
def test_exact_force_sum_matches_oracle(storage, lattice):
    """LBM_FORCE_SUM_EXACT: the same per-link terms summed in 128-bit
    integers; forces, torques and populations within the storage's bars."""
    case = GEOM_CASES[1]
    lat, ps = W.tiny_case(case["seed"], dims=case["dims"], periodic=case["periodic"],
                          n_particles=case["n_particles"], diameter_range=(4.0, 7.0),
                          speed=0.06, spin=0.006, u0=(0.02, -0.01, 0.005))
    r = _run(lat, ps, storage, 6, exact_forces=True, tag="exact", lattice=lattice)
    assert r["pop_err"] <= POP_TOL[storage] and r["F"] <= FORCE_TOL[storage] \
        and r["T"] <= FORCE_TOL[storage], r


def _force_series(lat, ps, steps, exact):
    gpu = B.Lattice.for_particles(lat, ps, storage="f32", treatments=11, exact_forces=exact)
    parts = B.DeviceParticles(ps)
    out = []
    for n in range(steps):
        parts.set_state(W.prescribed_state(ps, lat, float(n)))
        gpu.classify(parts)
        gpu.step(parts)
        F, T = gpu.forces()
        out.append(np.concatenate([F.cpu().numpy(), T.cpu().numpy()], 1))
    geo = (gpu.owner(), gpu.links(), gpu.refill())
    gpu.close()
    return np.array(out), geo


def test_exact_force_sum_repeats_bit_for_bit():
    """Sixty bodies on a 128^3 lattice, hundreds of link workgroups per body:
    two contexts give the same owners, links and refill set, and with exact
    sums the same force and torque bits every step (the link
    lists' order comes from atomics and differs between them).  The FP64
    atomic sums differ from them by their own rounding, which the cancellation
    between a body's link terms (each ~0.1, the net force ~1e-4) magnifies
    relative to the force: bounded here far inside the FP32 storage bar."""
    lat, ps, _ = W.config_c3(n_particles=60, n=128)
    a, ga = _force_series(lat, ps, 3, True)
    b, gb = _force_series(lat, ps, 3, True)
    c, _ = _force_series(lat, ps, 3, False)
    assert np.array_equal(a, b)
    # the geometry of the last classification repeats too (lists compared in
    # canonical order; their order in memory comes from atomics)
    assert np.array_equal(ga[0], gb[0])
    for k in ga[1]:
        assert np.array_equal(ga[1][k].view(np.uint8), gb[1][k].view(np.uint8)), k
    assert np.array_equal(ga[2][0], gb[2][0]) and np.array_equal(ga[2][1], gb[2][1])
    scale = np.abs(c).max(axis=(0, 2), keepdims=True)
    err = (np.abs(a - c) / scale).max()
    print(f"exact vs atomic sums: largest difference {err:.3e} of the body's force scale")
    assert err <= 1e-8, err
