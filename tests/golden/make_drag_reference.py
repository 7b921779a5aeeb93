"""Write the FP64 oracle's force and torque series for the replay runs of
paper_2206_11634_amd.workloads.drag_case, which the benchmark and the GPU tests
compare the HIP path against.

    python tests/golden/make_drag_reference.py [c1 c2 c3 c4]

Calls only the oracle (and the input generators).  Each case goes to
drag_<case>.npz here: F and T of shape (steps, bodies, 3), the fingerprint of
the run's inputs, and for c4 the sampled bodies, whose forces come from
sub-box runs of the oracle (tests/oracle_windows.py: the sub-box faces act
as walls, and with margins of 2 K + 4 nodes the sampled body's forces over
K steps equal those on the whole lattice)."""
from __future__ import annotations

import sys
import time
from pathlib import Path

import numpy as np

HERE = Path(__file__).resolve().parent
ROOT = HERE.parents[1]
for p in (str(ROOT), str(ROOT / "tests")):
    if p not in sys.path:
        sys.path.insert(0, p)

from oracle import oracle as O  # noqa: E402
from paper_2206_11634_amd import workloads as W  # noqa: E402

C4_MARGIN = 2 * 3 + 4


def whole_lattice(name):
    lat, ps, steps, treat, desc = W.drag_case(name)
    ora = O.Oracle(lat, treat=treat)
    F = np.zeros((steps, ps.n, 3))
    T = np.zeros((steps, ps.n, 3))
    t0 = time.time()
    for n in range(steps):
        P = W.prescribed_state(ps, lat, float(n))
        ora.classify(P)
        F[n], T[n] = ora.step(P)
        if n % 100 == 0:
            print(f"{name}: step {n}/{steps}, {time.time() - t0:.0f} s", flush=True)
    return dict(F=F, T=T, fingerprint=W.fingerprint(lat, ps, steps, treat), description=desc,
                oracle_threads=O.num_threads())


def c4_windows():
    import oracle_windows as OW
    lat, ps, steps, treat, desc = W.drag_case("c4")
    half_extra = 2 + C4_MARGIN
    sample = OW.sample_bodies(lat, ps, half_extra)
    traj = [W.prescribed_state(ps, lat, float(t)) for t in range(steps + 1)]
    F = np.zeros((steps, len(sample), 3))
    T = np.zeros((steps, len(sample), 3))
    for si, p in enumerate(sample):
        Fo, To, *_ = OW.run_window(lat, ps, traj, p, steps, half_extra, treat=treat)
        F[:, si], T[:, si] = Fo, To
        print(f"c4: body {p} done", flush=True)
    return dict(F=F, T=T, bodies=np.array(sample, np.int64),
                fingerprint=W.fingerprint(lat, ps, steps, treat), description=desc,
                oracle_threads=O.num_threads())


def main(names):
    for name in names:
        res = c4_windows() if name == "c4" else whole_lattice(name)
        out = HERE / f"drag_{name}.npz"
        np.savez(out, **{k: np.asarray(v) for k, v in res.items()})
        print(f"wrote {out}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or list(W.DRAG_CASES))
