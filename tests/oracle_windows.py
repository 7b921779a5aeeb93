"""Sub-box runs of the FP64 oracle around one body of a large lattice.

The oracle runs a non-periodic sub-box [lo, hi) holding every body whose
bounding ball reaches into it, translated by -lo (an exact FP64 operation for
coordinates inside the sub-box, so M, q and the owner tests see the same
values as on the whole lattice).  Faces of the sub-box that are not walls of
the lattice act as walls; their effect travels at most two nodes per step
(one by streaming, one through the x_ff of a link), so the body's forces and
the populations in the core of the sub-box equal those of the whole lattice
for as many steps as the margins allow."""
import numpy as np

from oracle import oracle as O
from paper_2206_11634_amd import workloads as W


subset = W.subset


def sample_bodies(lat, ps, half_extra):
    """Bodies whose sub-box stays inside the periodic axes: the lowest, the
    highest and two middle ones along the wall-normal axis z."""
    dims = np.array(lat.dims)
    ok = []
    for p in range(ps.n):
        h = int(np.ceil(ps.radius[p])) + half_extra
        c = np.floor(ps.pos[p]).astype(int)
        if all(c[a] - h >= 0 and c[a] + h + 1 <= dims[a] for a in range(3) if lat.periodic[a]):
            ok.append(p)
    ok = np.array(ok)
    z = ps.pos[ok, 2]
    order = ok[np.argsort(z)]
    return [int(order[0]), int(order[1]), int(order[len(order) // 2]), int(order[-1])]


def window(lat, ps, p, half_extra):
    dims = np.array(lat.dims)
    h = int(np.ceil(ps.radius[p])) + half_extra
    c = np.floor(ps.pos[p]).astype(int)
    lo, hi = c - h, c + h + 1
    real = np.zeros((3, 2), bool)   # faces that are the lattice's own walls
    for a in range(3):
        if not lat.periodic[a]:
            if lo[a] <= 0:
                lo[a], real[a, 0] = 0, True
            if hi[a] >= dims[a]:
                hi[a], real[a, 1] = dims[a], True
    return lo, hi, real



def run_window(lat, ps, traj, p, steps, half_extra, treat=O.TREAT_VIBB | O.TREAT_MISSING):
    """Oracle over a sub-box around body p for `steps` steps of the trajectory
    traj (list of global particle states) with treatment bits treat.  Returns
    the force and torque of p per step, the oracle, lo, the sub-box dims and
    its wall faces."""
    lo, hi, real = window(lat, ps, p, half_extra)
    wdims = hi - lo
    wlat, _, near = W.subbox(lat, ps, lo, hi)
    local = near.index(p)
    ora = O.Oracle(wlat, treat=treat)
    Fo, To = [], []
    for t in range(steps):
        P = subset(traj[t], near, -lo.astype(float))
        ora.classify(P)
        F, T = ora.step(P)
        Fo.append(F[local].copy())
        To.append(T[local].copy())
    return np.array(Fo), np.array(To), ora, lo, wdims, real


def core_fluid_nodes(lat, ora, lo, wdims, real, depth):
    """Fluid nodes of the sub-box at least `depth` nodes from its artificial
    faces: (sub-box indices, whole-lattice indices)."""
    dims = np.array(lat.dims)
    core_lo = np.where(real[:, 0], 0, depth)
    core_hi = wdims - np.where(real[:, 1], 0, depth)
    zz, yy, xx = np.meshgrid(*[np.arange(core_lo[a], core_hi[a]) for a in (2, 1, 0)],
                             indexing="ij")
    xx, yy, zz = xx.ravel(), yy.ravel(), zz.ravel()
    lnode = xx + wdims[0] * (yy + wdims[1] * zz)
    fl = ora.owner[lnode] == 0
    g = [(c[fl] + lo[a]) for a, c in enumerate((xx, yy, zz))]
    return lnode[fl], g[0] + dims[0] * (g[1] + dims[1] * g[2])
