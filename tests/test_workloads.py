"""Synthetic inputs: the sedimentation layout places every body clear of the
walls and of the other bodies (checked on the lattice nodes, independently of
the placement's own surface sampling)."""
import numpy as np

from paper_2206_11634_amd import workloads as W


def _solid_nodes(ps, p, dims, periodic):
    """Nodes with M_p >= c0_p (Eq. metaball), wrapped on periodic axes."""
    a, b = ps.ctrl_off[p], ps.ctrl_off[p + 1]
    c, r = ps.pos[p], ps.radius[p]
    lo, hi = np.floor(c - r - 1).astype(int), np.ceil(c + r + 1).astype(int)
    X, Y, Z = np.meshgrid(*[np.arange(lo[k], hi[k] + 1) for k in range(3)], indexing="ij")
    P = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
    M = np.zeros(len(P))
    for i in range(a, b):
        d = P - ps.world_pts[i]
        M += ps.K[i] / (d * d).sum(1)
    S = P[M >= ps.c0[p]]
    for k in range(3):
        if periodic[k]:
            S[:, k] %= dims[k]
    return S


def test_sedimentation_bodies_clear_of_walls_and_each_other():
    lat, ps, meta = W.config_c4(seed=9, n=96, per_axis=3)
    dims, per = lat.dims, lat.periodic
    sets = []
    for p in range(ps.n):
        S = _solid_nodes(ps, p, dims, per)
        assert len(S) > 0.5 * ps.volume[p]
        # walls in z at -0.5 and nz - 0.5: no solid node on the first or last layer
        assert S[:, 2].min() >= 1 and S[:, 2].max() <= dims[2] - 2, p
        sets.append(set(map(tuple, S.tolist())))
    for i in range(ps.n):
        for j in range(i + 1, ps.n):
            assert not (sets[i] & sets[j]), (i, j)
    assert meta["treatments"] == 11
