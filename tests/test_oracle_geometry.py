"""Pins of the oracle's coupling geometry (Sec. 2.3.1): node classification,
link sets with q (Eq. appq), and the refill set, against brute force written
independently here, and q against the exact surface crossing."""
import itertools

import numpy as np
import pytest

from oracle import oracle as O
from paper_2206_11634_amd import workloads as W

E19 = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
       (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1), (1, 0, -1),
       (-1, 0, 1), (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)]


def _M(pts, K, X):
    # ordered sum, r2 = (dx*dx + dy*dy) + dz*dz, as the convention fixes
    m = 0.0
    for p, k in zip(pts, K):
        dx, dy, dz = X[0] - p[0], X[1] - p[1], X[2] - p[2]
        m = m + k / ((dx * dx + dy * dy) + dz * dz)
    return m


def _image(c, L, per, center):
    if not per:
        return float(c)
    w = c % L
    d = w - center
    if d > 0.5 * L:
        return float(w - L)
    if d < -0.5 * L:
        return float(w + L)
    return float(w)


def brute_owner(lat, ps):
    dims, per = lat.dims, lat.periodic
    own = np.zeros(lat.ncell, np.int32)
    for k, j, i in itertools.product(range(dims[2]), range(dims[1]), range(dims[0])):
        for p in range(ps.n):
            a, b = ps.ctrl_off[p], ps.ctrl_off[p + 1]
            X = [_image(c, L, pr, ps.pos[p][ax])
                 for ax, (c, L, pr) in enumerate(zip((i, j, k), dims, per))]
            if _M(ps.world_pts[a:b], ps.K[a:b], X) >= ps.c0[p]:
                own[i + dims[0] * (j + dims[1] * k)] = p + 1
                break
    return own


def brute_links(lat, ps, own, treat=3):
    dims, per = lat.dims, lat.periodic
    nx, ny = dims[0], dims[1]

    def inside(c):
        out = []
        for v, L, pr in zip(c, dims, per):
            if 0 <= v < L:
                out.append(v)
            elif pr:
                out.append(v % L)
            else:
                return None
        return out

    def idx(c):
        return c[0] + nx * (c[1] + ny * c[2])

    recs = []
    for p in range(ps.n):
        a, b = ps.ctrl_off[p], ps.ctrl_off[p + 1]
        P, K = ps.world_pts[a:b], ps.K[a:b]
        for xs in np.nonzero(own == p + 1)[0]:
            cs = [xs % nx, (xs // nx) % ny, xs // (nx * ny)]
            Xs = [_image(cs[ax], dims[ax], per[ax], ps.pos[p][ax]) for ax in range(3)]
            Ms = _M(P, K, Xs)
            for d in range(1, 19):
                e = E19[d]
                raw = [cs[ax] - e[ax] for ax in range(3)]
                cn = inside(raw)
                if cn is not None and own[idx(cn)] == p + 1:
                    continue
                Xn = [_image(raw[ax], dims[ax], per[ax], ps.pos[p][ax]) for ax in range(3)]
                Mn = _M(P, K, Xn)
                if cn is not None and own[idx(cn)] == 0:
                    cff = inside([cn[ax] - e[ax] for ax in range(3)])
                    ff = cff is not None and own[idx(cff)] == 0
                    kind = 0 if (ff and (treat & 1)) else 1
                else:
                    if not (treat & 2) or not (Mn < ps.c0[p]):
                        continue
                    kind = 2
                recs.append((xs, d, kind, p, (ps.c0[p] - Mn) / (Ms - Mn)))
    return recs


CASES = [
    dict(seed=1, dims=(12, 10, 9), periodic=(1, 0, 1), n_particles=3),
    dict(seed=2, dims=(11, 12, 10), periodic=(1, 1, 1), n_particles=2),
    dict(seed=3, dims=(10, 9, 12), periodic=(0, 0, 0), n_particles=3),
    dict(seed=4, dims=(14, 12, 10), periodic=(0, 1, 0), n_particles=4),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"seed{c['seed']}")
def test_classification_and_links_bruteforce(case):
    lat, ps = W.tiny_case(case["seed"], dims=case["dims"], periodic=case["periodic"],
                          n_particles=case["n_particles"], diameter_range=(3.0, 5.0))
    o = O.Oracle(lat)
    own = o.owners(ps)
    ref_own = brute_owner(lat, ps)
    assert np.array_equal(own, ref_own)
    assert (own > 0).sum() > 0
    L = o.build_links(ps, own)
    ref = brute_links(lat, ps, ref_own)
    assert len(L) == len(ref)
    assert np.array_equal(L.node, [r[0] for r in ref])
    assert np.array_equal(L.d, [r[1] for r in ref])
    assert np.array_equal(L.kind, [r[2] for r in ref])
    assert np.array_equal(L.part, [r[3] for r in ref])
    assert np.array_equal(L.q.view(np.uint64), np.array([r[4] for r in ref]).view(np.uint64))
    assert np.all((L.q > 0) & (L.q <= 1))


def test_links_cover_wrap_walls_and_gaps():
    """The tiny cases exercise every link kind, including missing force points."""
    kinds = np.zeros(3, int)
    for case in CASES:
        lat, ps = W.tiny_case(case["seed"], dims=case["dims"], periodic=case["periodic"],
                              n_particles=case["n_particles"], diameter_range=(3.0, 5.0))
        o = O.Oracle(lat)
        o.classify(ps)
        kinds += np.bincount(o.links.kind, minlength=3)
        # every link that reconstructs writes ghost slot d-bar of its solid
        # node x_s, and that slot is pulled by x_s - e_d alone: no two
        # writing links share a (node, d)
        w = o.links.kind != 2
        key = o.links.node[w].astype(np.int64) * 32 + o.links.d[w]
        assert np.unique(key).size == key.size
    assert np.all(kinds > 0), kinds


def test_refill_set_is_solid_then_fluid():
    lat, ps = W.tiny_case(5, dims=(14, 12, 12), periodic=(1, 1, 1), n_particles=2,
                          speed=0.4, spin=0.05)
    o = O.Oracle(lat)
    o.classify(ps)
    own0 = o.owner.copy()
    o.step(ps)
    p1 = W.prescribed_state(ps, lat, 1.0)
    o.classify(p1)
    expect = np.nonzero((own0 > 0) & (o.owner == 0))[0]
    assert len(expect) > 0
    assert np.array_equal(o.refill_nodes, expect)


def test_q_linear_interpolation_of_M():
    """Eq. appq is the zero of the straight line through (0, M(x_n)) and
    (1, M(x_s)) at level c0; checked with numpy's interpolation."""
    lat, ps = W.tiny_case(6, dims=(14, 13, 12), periodic=(1, 1, 1), n_particles=3)
    o = O.Oracle(lat)
    o.classify(ps)
    L = o.links
    nx, ny = lat.nx, lat.ny
    for l in range(0, len(L), 7):
        p, xs, d = L.part[l], L.node[l], L.d[l]
        a, b = ps.ctrl_off[p], ps.ctrl_off[p + 1]
        cs = [xs % nx, (xs // nx) % ny, xs // (nx * ny)]
        Xs = np.array([_image(cs[ax], lat.dims[ax], lat.periodic[ax], ps.pos[p][ax])
                       for ax in range(3)])
        Xn = Xs - np.array(E19[d])
        Ms = O.metaball(ps.world_pts[a:b], ps.K[a:b], Xs)
        Mn = O.metaball(ps.world_pts[a:b], ps.K[a:b], Xn)
        q_ref = np.interp(ps.c0[p], [Mn, Ms], [0.0, 1.0])
        assert abs(L.q[l] - q_ref) < 1e-13


def test_q_sphere_against_exact_crossing():
    """For a sphere the surface crossing along a link solves a quadratic; the
    linear approximation of Eq. appq stays in (0, 1] and is within a few
    percent on average (the paper reports about 5% relative error)."""
    sh = W.sphere_shape(15.0, 0.1)
    lat = W.LatticeSpec(24, 24, 24, (1, 1, 1))
    ps = W.make_particles([sh], [12.3, 11.8, 12.1], [1, 0, 0, 0], 1.0)
    o = O.Oracle(lat)
    o.classify(ps)
    L = o.links
    r = 7.5
    errs = []
    for l in range(len(L)):
        xs, d = L.node[l], L.d[l]
        cs = np.array([xs % 24, (xs // 24) % 24, xs // 576], float)
        e = np.array(E19[d], float)
        xn = cs - e - ps.pos[0]
        # |xn + t e|^2 = r^2, smallest root in [0, 1]
        a, b, c = e @ e, 2 * xn @ e, xn @ xn - r * r
        t = (-b - np.sqrt(b * b - 4 * a * c)) / (2 * a)
        assert -1e-12 <= t <= 1 + 1e-12
        errs.append(abs(L.q[l] - t) / max(t, 1e-3))
    errs = np.array(errs)
    assert np.all((L.q > 0) & (L.q <= 1))
    assert 0.005 < np.median(errs) < 0.1, np.median(errs)


def test_exact_q_sphere_matches_the_quadratic_root():
    """With treatment bit 4, q solves Eq. calq; for a sphere that root is the
    smaller root of |x_n + q e - x_p|^2 = r^2 (r = sqrt(K / c0)), which the
    Newton iteration must reach to rounding.  Links keep their kinds and
    nodes; only q changes."""
    sh = W.sphere_shape(15.0, 0.1)
    lat = W.LatticeSpec(24, 24, 24, (1, 1, 1))
    ps = W.make_particles([sh], [12.3, 11.8, 12.1], [1, 0, 0, 0], 1.0)
    lin = O.Oracle(lat).classify(ps).links
    ex = O.Oracle(lat, treat=O.TREAT_VIBB | O.TREAT_MISSING | O.TREAT_EXACT_Q).classify(ps).links
    assert np.array_equal(lin.node, ex.node) and np.array_equal(lin.d, ex.d)
    assert np.array_equal(lin.kind, ex.kind)
    r = np.sqrt(sh.K[0] / sh.c0)
    worst = 0.0
    for l in range(len(ex)):
        xs, d = ex.node[l], ex.d[l]
        cs = np.array([xs % 24, (xs // 24) % 24, xs // 576], float)
        e = np.array(E19[d], float)
        xn = cs - e - ps.pos[0]
        a, b, c = e @ e, 2 * xn @ e, xn @ xn - r * r
        t = (-b - np.sqrt(b * b - 4 * a * c)) / (2 * a)
        worst = max(worst, abs(ex.q[l] - t))
    assert worst < 1e-12, worst
    assert np.all((ex.q >= 0) & (ex.q <= 1))


def test_exact_q_solves_calq_for_metaballs():
    """For multi-point metaballs: M(x_n + q e) = c0 at the returned q (to a
    relative 1e-12), and for bodies much larger than the lattice spacing the
    linear estimate of Eq. appq differs from it by a few percent on average,
    as the paper reports."""
    lat, ps = W.tiny_case(6, dims=(44, 42, 40), periodic=(1, 1, 1), n_particles=2,
                          diameter_range=(16.0, 20.0))
    lin = O.Oracle(lat).classify(ps).links
    ex = O.Oracle(lat, treat=O.TREAT_VIBB | O.TREAT_MISSING | O.TREAT_EXACT_Q).classify(ps).links
    nx, ny = lat.nx, lat.ny
    rel = []
    for l in range(len(ex)):
        p, xs, d = ex.part[l], ex.node[l], ex.d[l]
        a, b = ps.ctrl_off[p], ps.ctrl_off[p + 1]
        cs = [xs % nx, (xs // nx) % ny, xs // (nx * ny)]
        Xs = np.array([_image(cs[ax], lat.dims[ax], lat.periodic[ax], ps.pos[p][ax])
                       for ax in range(3)])
        Xn = Xs - np.array(E19[d])
        M = _M(ps.world_pts[a:b], ps.K[a:b], Xn + ex.q[l] * np.array(E19[d], float))
        assert abs(M - ps.c0[p]) <= 1e-12 * ps.c0[p], (l, M, ps.c0[p])
        rel.append(abs(lin.q[l] - ex.q[l]) / max(ex.q[l], 1e-3))
    assert 0.003 < np.median(rel) < 0.1, np.median(rel)
