"""Timing of dem_step on jittered sphere packs (every body in contact).

    python -m paper_2206_11634_amd.dem_pack_bench [--sizes 14x13,20x20,30x30]

Spheres of diameter 5.2 sit on a 5-unit lattice (n x n columns of m layers,
Gaussian jitter 0.15) in a box periodic in x and y with walls in z, moving
with seeded velocities; each call is 10 substeps of 0.1.  Packs of 2048
particles and more take the cell-grid broad phase; the 1000-metaball
sedimentation workload is timed beside them (all-pairs broad phase).  Prints
one line per pack: particles and milliseconds per call."""
import argparse
import time

import numpy as np


def sphere_pack(nx: int, nz: int, seed: int = 21):
    from paper_2206_11634_amd import workloads as W
    rng = np.random.default_rng(seed)
    L = max(5 * nx, 5 * nz + 8)
    lat = W.LatticeSpec(L, L, L, (1, 1, 0), tau=0.6)
    g = (np.arange(nx) + 0.5) * 5.0
    z = 4.0 + 5.0 * np.arange(nz)
    X, Y, Z = np.meshgrid(g, g, z, indexing="ij")
    pos = np.stack([X.ravel(), Y.ravel(), Z.ravel()], -1)
    pos = pos + rng.normal(size=pos.shape) * 0.15
    n = len(pos)
    quats = np.array([W.random_quaternion(rng) for _ in range(n)])
    ps = W.make_particles([W.sphere_shape(5.2, 0.1)] * n, pos, quats, 1.5)
    ps.vel = rng.normal(size=(n, 3)) * 0.02
    ps.omega = rng.normal(size=(n, 3)) * 0.002
    return lat, ps


def time_dem(lat, ps, gravity=(0.0, 0.0, -1e-4), calls: int = 20) -> float:
    import torch
    from paper_2206_11634_amd import binding as B
    from paper_2206_11634_amd import workloads as W
    gpu = B.Lattice.for_particles(lat, ps, storage="f32")
    parts = B.DeviceParticles(ps)
    prm = B.DemParams.make(**W.dem_defaults(ps, gravity=gravity))
    for _ in range(3):
        gpu.dem(parts, 10, 0.1, prm)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(calls):
        gpu.dem(parts, 10, 0.1, prm)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t) / calls * 1e3
    gpu.sync()
    gpu.close()
    return ms


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--sizes", default="14x13,20x20,30x30",
                    help="packs as columns-per-side x layers")
    args = ap.parse_args()
    from paper_2206_11634_amd import workloads as W
    lat, ps, meta = W.config_c4()
    print(f"c4 metaballs: {ps.n} particles, {time_dem(lat, ps, meta['gravity']):.3f} ms per call",
          flush=True)
    for item in args.sizes.split(","):
        nx, nz = (int(v) for v in item.split("x"))
        lat, ps = sphere_pack(nx, nz)
        print(f"sphere pack {nx}x{nx}x{nz}: {ps.n} particles, {time_dem(lat, ps):.3f} ms per call",
              flush=True)


if __name__ == "__main__":
    main()
