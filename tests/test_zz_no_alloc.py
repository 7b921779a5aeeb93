"""dem_step_noalloc, the allocation-free variant of dem_step (its work space
in a static device array), against dem_step through the C-ABI: two calls in a
row, the second on a context with fewer particles, each compared with
dem_step on a twin context fed the same inputs."""
import numpy as np
import pytest

from paper_2206_11634_amd import binding as B
from paper_2206_11634_amd import workloads as W

pytestmark = pytest.mark.gpu


def _bodies(n, seed):
    """n spheres and metaballs in a box with walls in z, packed so that pairs
    and walls come into contact within the call."""
    rng = np.random.default_rng(seed)
    lat = W.LatticeSpec(64, 48, 40, (1, 1, 0))
    shapes, pos = [], []
    for k in range(n):
        if k % 2:
            pts = np.array([[0.0, 0, 0], [1.0, 0, 0], [0.5, 0.7, 0]])
            shapes.append(W.metaball_shape(pts, rng.uniform(0.5, 1.5, 3) * 0.2, 0.3, d_eq=9.0,
                                           samples_per_unit=3.0))
        else:
            shapes.append(W.sphere_shape(9.0, 0.3))
        pos.append([8.0 + 9.2 * k, 24.0 + rng.uniform(-1, 1), 4.3 + rng.uniform(0, 0.2)])
    quats = [W.random_quaternion(rng) for _ in range(n)]
    vel = rng.normal(size=(n, 3)) * 0.02
    vel[:, 2] -= 0.01
    ps = W.make_particles(shapes, pos, quats, 1.5, vel=vel,
                          omega=rng.normal(size=(n, 3)) * 0.005)
    return lat, ps


def _run(lat, ps, noalloc, prm, calls):
    gpu = B.Lattice.for_particles(lat, ps, storage="f64")
    parts = B.DeviceParticles(ps)
    for _ in range(calls):
        (gpu.dem_noalloc if noalloc else gpu.dem)(parts, 10, 0.1, prm)
    gpu.sync()
    state = gpu.dem_checkpoint().cpu().numpy()
    out = parts.to_host(ps)
    gpu.close()
    return out, state


def _dem_state(raw, n, slots=32):
    """The DEM checkpoint: pair records by (particle, partner) (slot numbers
    depend on the order in which threads claimed them), wall records,
    contact sums."""
    b = raw.tobytes()
    o_key = n * slots * 8 * 8
    o_pw = o_key + n * slots * 4
    o_fc = o_pw + n * 6 * 8 * 8
    pp = np.frombuffer(b, np.float64, n * slots * 8, 0).reshape(n, slots, 8)
    key = np.frombuffer(b, np.int32, n * slots, o_key).reshape(n, slots)
    pw = np.frombuffer(b, np.float64, n * 6 * 8, o_pw).reshape(n, 6, 8)
    fc = np.frombuffer(b, np.float64, n * 6, o_fc).reshape(n, 6)
    # a key is the partner's index + 1; 0 marks a free slot
    recs = {(i, int(key[i, s]) - 1): pp[i, s] for i in range(n) for s in range(slots)
            if key[i, s] > 0}
    return recs, pw, fc


def _close(a, b):
    return np.abs(a - b).max() <= 1e-12 * max(1.0, np.abs(b).max())


def test_dem_step_noalloc_matches_dem_step_on_two_calls():
    for n, seed in ((6, 3), (3, 4)):   # the second call has fewer particles
        lat, ps = _bodies(n, seed)
        kw = W.dem_defaults(ps, gravity=(0.0, 0.0, -2e-4))
        prm = B.DemParams.make(**kw)
        ref, st_ref = _run(lat, ps, False, prm, 25)
        got, st_got = _run(lat, ps, True, prm, 25)
        for k in ("pos", "vel", "omega", "quat", "world_pts"):
            assert _close(getattr(got, k), getattr(ref, k)), (n, k)
        assert np.abs(ref.pos - ps.pos).max() > 1e-3
        rr, pw_r, fc_r = _dem_state(st_ref, n)
        rg, pw_g, fc_g = _dem_state(st_got, n)
        assert rr.keys() == rg.keys(), n
        for key in rr:
            assert _close(rg[key], rr[key]), (n, key)
        assert _close(pw_g, pw_r) and _close(fc_g, fc_r), n
        # contacts happened: with walls (the bodies start on the floor) and pairs
        assert np.abs(pw_r[:, :, 0]).max() == 1.0
        assert any(r[0] == 1.0 for r in rr.values()), n
