"""The sub-box runs used for sampled parity on the 512^3 workload reproduce the
whole-lattice oracle: forces of the sampled bodies and populations in the core
of each sub-box, over the steps the margins cover (a 96^3 lattice with the
same layout, 27 bodies, walls in z, moving bodies so that nodes are
refilled)."""
import numpy as np

import oracle_windows as OW
from oracle import oracle as O
from paper_2206_11634_amd import workloads as W

K = 3


def test_sub_box_runs_equal_the_whole_lattice():
    lat, ps, meta = W.config_c4(seed=9, n=96, per_axis=3)
    rng = np.random.default_rng(3)
    ps.vel = rng.normal(size=(ps.n, 3)) * 0.03
    ps.omega = rng.normal(size=(ps.n, 3)) * 0.003
    traj = [W.prescribed_state(ps, lat, float(t)) for t in range(K + 1)]
    half_extra = 2 + 2 * K + 4
    sample = OW.sample_bodies(lat, ps, half_extra)
    full = O.Oracle(lat)
    F, T = [], []
    refilled = 0
    for t in range(K):
        full.classify(traj[t])
        refilled += len(full.refill_nodes)
        f, tq = full.step(traj[t])
        F.append(f.copy())
        T.append(tq.copy())
    F, T = np.array(F), np.array(T)
    assert refilled > 0
    walls_seen = 0
    for p in sample:
        Fo, To, ora, lo, wdims, real = OW.run_window(lat, ps, traj, p, K, half_extra)
        walls_seen += int(real.any())
        assert np.abs(Fo - F[:, p]).max() <= 1e-13 * np.abs(F[:, p]).max()
        assert np.abs(To - T[:, p]).max() <= 1e-13 * np.abs(T[:, p]).max()
        lnode, gnode = OW.core_fluid_nodes(lat, ora, lo, wdims, real, 2 * K + 2)
        assert len(lnode) > 1000
        assert np.array_equal(full.owner[gnode], np.zeros(len(gnode), full.owner.dtype))
        assert np.abs(ora.f[:, lnode] - full.f[:, gnode]).max() <= 1e-15
    assert walls_seen >= 1
