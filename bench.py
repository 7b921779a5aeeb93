#!/usr/bin/env python3
"""Throughput of the coupled sharp-interface metaball LBM step on one MI355X.

One step = lbm_classify_nodes (FP64 classification, links, refill) +
lbm_step (VIBB / halfway reconstruction, momentum exchange, fused
stream-collide) + lbm_particle_forces + dem_step (FP64 metaball DEM,
sub-cycled), on the 512^3 sedimentation workload (1000 metaballs, 20% solids)
with synthetic seeded inputs.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "MLUPS + % HBM roofline (FP32/FP16-store vs plain), drag err; adjoint steps/s"

# HBM bytes per stream-collide launch measured with rocprofv3 FETCH_SIZE and
# WRITE_SIZE passes (scaled by a copy kernel of known size; see profiles/),
# valid only for the kernel source they were taken on.
MEASURED_TRAFFIC = {
    ("c4_sediment_512cube_1000p", "f32"): dict(source_sha256_16="a244481d9894da87",
                                              read=10.294e9, written=12.348e9),
}
HBM_PEAK_GBS = 8000.0
BYTES = {"f64": 8, "f32": 4, "f16": 2}


def run_storage(lat, ps, meta, storage, steps, warmup, profile=True, treatments=None, lattice=19,
                seq_steps=0):
    import torch
    from paper_2206_11634_amd import binding as B
    from paper_2206_11634_amd import workloads as W

    if treatments is None:   # the workload's own treatment bits
        treatments = int(meta.get("treatments", 3))
    gpu = B.Lattice.for_particles(lat, ps, storage=storage, treatments=treatments,
                                  lattice=lattice)
    parts = B.DeviceParticles(ps)
    prm = B.DemParams.make(**W.dem_defaults(ps, gravity=meta["gravity"]))
    n_sub = int(meta.get("n_sub", 10))
    gpu.classify(parts)

    def one_step(sync):
        # the link pass, then the stream-collide pass with the DEM sub-cycle
        # beside it (lbm_step_dem: the same results as lbm_step, dem_step)
        gpu.step_dem(parts, n_sub, 1.0 / n_sub, prm)
        gpu.forces()
        # timed steps classify without the host read-back of list counts
        # (lbm_classify_nodes_async); the warm-up steps, which read them back,
        # sized the lists, and the check after the loop reports anything the
        # timed classifications latched
        gpu.classify(parts, sync=sync)

    for _ in range(warmup):
        one_step(True)
    torch.cuda.synchronize()
    if profile:
        gpu.profile(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        one_step(False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gpu.sync()   # raises on a latched overflow, rejected particle or non-finite force
    prof = gpu.profile_read() if profile else {}
    if profile:
        gpu.profile(False)
    seq = None
    if seq_steps:
        # after the timed steps: lbm_step, the forces and dem_step one after
        # the other, so that the stream-collide pass has the chip to itself
        gpu.profile(True)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        for _ in range(seq_steps):
            gpu.step(parts)
            gpu.forces()
            gpu.dem(parts, n_sub, 1.0 / n_sub, prm)
            gpu.classify(parts, sync=False)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        gpu.sync()
        seq = dict(ms_per_step=(t3 - t2) * 1e3 / seq_steps, prof=gpu.profile_read())
        gpu.profile(False)
    n_solid = int(torch.count_nonzero(gpu.flag[: gpu.ncell]).item())
    counts = gpu.classify(parts)
    gpu.close()
    del gpu, parts
    torch.cuda.empty_cache()
    ms = (t1 - t0) * 1e3 / steps
    return dict(ms_per_step=ms, n_solid=n_solid, prof=prof, n_links=int(counts.n_links),
                n_refill=int(counts.n_refill), n_cand=int(counts.n_candidates), seq=seq)


def _stream_source_hash():
    """Hash of the source the stream-collide kernel is compiled from: the
    kernel's own text, its workgroup-to-node mapping, the storage traits and
    stencil headers, and the Geom and Phys records it takes."""
    import hashlib
    import re
    csrc = os.path.join(ROOT, "paper_2206_11634_amd", "csrc")

    def read(name):
        with open(os.path.join(csrc, name), encoding="utf-8") as fh:
            return fh.read()

    stream = read("lbm_stream.hip")
    k = re.search(r"template <int S>\n__global__[^\n]*k_stream_collide\(.*?\n}\n", stream, re.S)
    m = re.search(r"__device__ __forceinline__ uint32_t xcd_block\(\).*?\n}\n", stream, re.S)
    internal = read("lbm_internal.h")
    parts = [k.group(0) if k else stream, m.group(0) if m else stream, read("lbm_kernels.h"),
             read("lbm_stencil.h")]
    for name in ("Geom", "Phys"):
        m = re.search(r"struct " + name + r" \{.*?\n\};", internal, re.S)
        parts.append(m.group(0) if m else internal)
    h = hashlib.sha256()
    for part in parts:
        h.update(part.encode())
    return h.hexdigest()[:16]


def bulk_roofline(res, lat, storage, workload=None, Q=19):
    """Algorithmic bytes of one stream-collide launch, per cell update of the
    lattice: 2 Q s + 1 bytes (Q = 19 populations of s bytes read and written,
    plus the 1-byte flag), times every cell of the lattice.  Also reported: the
    stricter count of what the method needs, every fluid node reading and
    writing 19 populations and writing its moments (rho - 1, u), every node
    its flag, solid nodes nothing."""
    ncell = lat.ncell
    nfluid = ncell - res["n_solid"]
    per_cell = 2 * Q * BYTES[storage] + 1
    bytes_launch = ncell * per_cell
    per_fluid = 2 * Q * BYTES[storage] + 4 * BYTES[storage]
    bytes_fluid = nfluid * per_fluid + ncell * 1
    ms, n = res["prof"]["bulk"]
    avg_ms = ms / max(n, 1)
    achieved = bytes_launch / (avg_ms * 1e-3) / 1e9
    traffic = None
    rec = MEASURED_TRAFFIC.get((workload, storage)) if Q == 19 else None
    if rec and rec["source_sha256_16"] == _stream_source_hash():
        traffic = int(rec["read"] + rec["written"])
    return dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic,
                kernel="k_stream_collide", avg_ms=round(avg_ms, 4),
                bytes_per_launch=int(bytes_launch), bytes_per_cell=per_cell,
                fluid_only=dict(bytes_per_launch=int(bytes_fluid), bytes_per_fluid_cell=per_fluid,
                                bytes_per_cell_flag=1,
                                achieved=round(bytes_fluid / (avg_ms * 1e-3) / 1e9, 1)))


def copy_ceiling(nbytes, reps=5):
    """Rate of a plain elementwise copy (out = in * 1) moving the same bytes
    as one stream-collide launch's populations, read and written once, timed
    with hipEvents: what HBM delivers to a streaming kernel on this device."""
    import torch
    n = int(nbytes // 4)
    a = torch.zeros(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.mul(a, 1.0, out=b)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        torch.mul(a, 1.0, out=b)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return round(2 * n * 4 / (ms * 1e-3) / 1e9, 1)


def cpu_baseline(seconds=12.0):
    """The FP64 oracle on a bounded sample of the timed workload: the sub-box
    [0, 128)^3 of the 512^3 sedimentation lattice (its z = 0 wall and the
    bodies reaching into it; the other faces act as walls), classify + step
    repeated for about `seconds`, on all of the host's threads and on one."""
    from oracle import oracle as O
    from paper_2206_11634_amd import workloads as W

    lat, ps, meta = W.config_c4()
    wlat, sub, near = W.subbox(lat, ps, (0, 0, 0), (128, 128, 128))
    threads = O.num_threads()

    def rate(nthreads):
        O.set_num_threads(nthreads)
        o = O.Oracle(wlat, treat=int(meta.get("treatments", 3)))
        o.classify(sub)
        steps = 0
        t0 = time.perf_counter()
        while True:
            o.step(sub)
            o.classify(sub)
            steps += 1
            if time.perf_counter() - t0 > seconds and steps >= 2:
                break
        dt = time.perf_counter() - t0
        return wlat.ncell * steps / dt / 1e6, steps, dt

    v_all, n_all, t_all = rate(threads)
    v_one, n_one, t_one = rate(1)
    O.set_num_threads(threads)
    return dict(value=round(v_all, 3), unit="MLUPS", cores=threads, kind="oracle",
                value_1thread=round(v_one, 3),
                sample=f"FP64 oracle classify+step on the sub-box [0,128)^3 of the 512^3 "
                       f"sedimentation lattice ({len(near)} bodies reaching into it, "
                       f"treatment bits {int(meta.get('treatments', 3))}): {n_all} steps in "
                       f"{t_all:.1f} s on {threads} threads, {n_one} steps in {t_one:.1f} s "
                       f"on 1 thread")


def _reference_series(name, lat, ps, steps, treat):
    """The oracle's stored force and torque series of a drag case
    (tests/golden/make_drag_reference.py), or None with the reason when it is
    missing or was made from other inputs."""
    from paper_2206_11634_amd import workloads as W
    path = os.path.join(ROOT, "tests", "golden", f"drag_{name}.npz")
    if not os.path.exists(path):
        return None, f"no oracle reference ({path})"
    d = np.load(path, allow_pickle=False)
    if str(d["fingerprint"]) != W.fingerprint(lat, ps, steps, treat):
        return None, "oracle reference made from other inputs"
    return d, None


def _replay(lat, ps, steps, treat, storage, bodies=None):
    """Force and torque of the GPU path on a prescribed replay, [steps, n, 6]."""
    import torch
    from paper_2206_11634_amd import binding as B
    from paper_2206_11634_amd import workloads as W

    traj = B.DeviceTrajectory([W.prescribed_state(ps, lat, float(n)) for n in range(steps + 1)])
    gpu = B.Lattice.for_particles(lat, ps, storage=storage, treatments=treat)
    F = torch.zeros((steps, ps.n, 6), dtype=torch.float64, device=gpu.device)
    for k in range(steps):
        gpu.classify(traj[k])
        gpu.step(traj[k])
        f, t = gpu.forces()
        F[k, :, :3] = f
        F[k, :, 3:] = t
    out = F.cpu().numpy()
    gpu.close()
    del gpu, traj
    torch.cuda.empty_cache()
    return out if bodies is None else out[:, bodies]


def _errors(g, F, T):
    """Per body: max over steps of |X_gpu - X_oracle| over the largest
    |X_oracle| of the run (vector norms), for force and torque; the largest and
    the median over the bodies."""
    res = {}
    for name, sl, ref in (("force", slice(0, 3), F), ("torque", slice(3, 6), T)):
        num = np.linalg.norm(g[:, :, sl] - ref, axis=2).max(0)
        den = np.linalg.norm(ref, axis=2).max(0)
        e = num / np.maximum(den, 1e-300)
        res[name] = dict(max=float(e.max()), median=float(np.median(e)))
    return res


DRAG_BAR = {"f64": 1e-10, "f32": 1e-4, "f16": 2e-2}


def drag_errors(storages=("f64", "f32", "f16")):
    """Force and torque of each storage against the FP64 oracle on the replay
    runs of every workload (workloads.drag_case): c1 (200 steps), c2 (2000
    steps), c3 (200 bodies, 100 steps) on the whole lattice, c4 on sampled
    bodies over 3 steps (the oracle's sub-box runs)."""
    from paper_2206_11634_amd import workloads as W

    out = {}
    for name in W.DRAG_CASES:
        lat, ps, steps, treat, desc = W.drag_case(name)
        ref, why = _reference_series(name, lat, ps, steps, treat)
        if ref is None:
            out[name] = dict(workload=desc, skipped=why)
            continue
        bodies = ref["bodies"] if "bodies" in ref.files else None
        res = dict(workload=desc, treatments=treat)
        for storage in storages:
            g = _replay(lat, ps, steps, treat, storage, bodies)
            e = _errors(g, ref["F"], ref["T"])
            e["within_bar"] = bool(max(e["force"]["max"], e["torque"]["max"]) <= DRAG_BAR[storage])
            res[storage] = e
        out[name] = res
        print(f"[bench] drag {name}: " + ", ".join(
            f"{st} {res[st]['force']['max']:.2e}" for st in storages), file=sys.stderr, flush=True)
    out["bars"] = DRAG_BAR
    out["measure"] = ("per body, max over steps |F_gpu - F_oracle| / max over steps |F_oracle| "
                      "(vector norms); max and median over the bodies")
    return out


def exact_q_effect(lat, ps, meta, steps=200):
    """q from Eq. calq (bracketed Newton) instead of Eq. appq: the drag change
    on the 40x40x80 sphere descent (FP32, prescribed motion), and the cost on
    the benchmark workload (classification phase, 5 steps)."""
    from paper_2206_11634_amd import binding as B
    from paper_2206_11634_amd import workloads as W

    l1, p1, _ = W.config_c1()
    p1.vel[:] = [0.0, 0.0, -0.01]
    p1.omega[:] = [0.0, 0.002, 0.0]
    traj = [W.prescribed_state(p1, l1, float(n)) for n in range(steps)]
    Fz = {}
    for name, treat in (("linear", 3), ("exact", 7)):
        gpu = B.Lattice.for_particles(l1, p1, storage="f32", treatments=treat)
        parts = B.DeviceParticles(p1)
        out = []
        for n in range(steps):
            parts.set_state(traj[n])
            gpu.classify(parts)
            gpu.step(parts)
            F, _ = gpu.forces()
            out.append(F[0].cpu().numpy().copy())
        gpu.close()
        Fz[name] = np.array(out)
    lin, ex = Fz["linear"], Fz["exact"]
    tail = slice(steps // 2, None)
    res = dict(
        drag_mean_rel_diff=float(abs(lin[tail, 2].mean() - ex[tail, 2].mean()) / abs(ex[tail, 2].mean())),
        force_series_rel_diff=float(np.abs(lin - ex).max() / np.abs(ex).max()),
        sphere_workload=f"c1 40x40x80 sphere d=10, prescribed descent 0.01 lu/step, {steps} steps, FP32")
    r = run_storage(lat, ps, meta, "f32", 5, 1, treatments=int(meta.get("treatments", 3)) | 4)
    res["ms_per_step"] = round(r["ms_per_step"], 4)
    res["classify_ms"] = round(r["prof"]["classify"][0] / max(r["prof"]["classify"][1], 1), 4)
    return res


def adjoint_bench(fd_check=True):
    """The differentiation form on the 128^3 channel: FP32 forward over 2000
    steps with checkpoints every 100, then the adjoint window by window
    (recomputation included), J = mean x-force on the particle; timed on a
    second pass.  With
    fd_check the gradient is compared with central differences of the FP64
    forward pass."""
    import torch
    from paper_2206_11634_amd import adjoint as AD
    from paper_2206_11634_amd import workloads as W

    lat, ps, meta = W.config_c5()
    T, K = meta["steps"], meta["checkpoint"]
    prob = AD.Problem(lat=lat, ps=ps, steps=T, window=K, storage=meta["storage"])
    v, F, tau = ps.vel.copy(), np.array(lat.body_force), lat.tau
    prob.initial()
    # a first pass allocates the checkpoints and the tape and times the
    # adjoint kernels with the library's event timers; the second, without
    # timers, gives the rates
    _, run = AD.forward(prob, v, F, tau, keep=True)
    stats = {}
    AD.backward(run, stats)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J, run = AD.forward(prob, v, F, tau, keep=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dv, dF, dtau = AD.backward(run)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    adj_ms, adj_n = stats.get("adjoint", (0.0, 0))
    out = dict(workload=meta["name"], lattice=[lat.nx, lat.ny, lat.nz], steps=T, checkpoint=K,
               storage=meta["storage"], J=J,
               forward_steps_per_s=round(T / (t1 - t0), 1),
               adjoint_steps_per_s=round(T / (t2 - t1), 1),
               adjoint_kernels_ms_per_step=round(adj_ms / max(adj_n, 1), 4),
               grad=dict(dJ_dU=dv[0].tolist(), dJ_dF=dF.tolist(), dJ_dtau=dtau))
    print(f"[bench] adjoint: forward {t1 - t0:.2f} s, backward {t2 - t1:.2f} s",
          file=sys.stderr, flush=True)
    if fd_check:
        import dataclasses
        ref = dataclasses.replace(prob, storage="f64")

        def fd(kind, h):
            def at(d):
                vv, FF, tt = v.copy(), F.copy(), tau
                if kind == "U":
                    vv[0, 0] += d
                elif kind == "F":
                    FF[0] += d
                else:
                    tt += d
                return AD.evaluate(ref, vv, FF, tt)
            return (at(h) - at(-h)) / (2 * h)

        g = dict(U_x=(dv[0, 0], fd("U", 1e-4)), F_x=(dF[0], fd("F", 1e-7)),
                 tau=(dtau, fd("tau", 1e-4)))
        out["fd_rel_err"] = {k: float(abs(a - b) / abs(b)) for k, (a, b) in g.items()}
        out["fd_reference"] = "central differences of the FP64-storage forward pass"
    out["free_motion"] = free_adjoint_bench(lat, ps, meta, fd_check)
    return out


def free_adjoint_bench(lat, ps, meta, fd_check=True):
    """The same channel with the particle moving freely (dem_step after every
    step, 10 substeps): forward and adjoint (through the DEM) steps per second
    and dJ/dv0_x against central differences of the FP64 free-motion pass."""
    import dataclasses
    import torch
    from paper_2206_11634_amd import adjoint as AD

    T, K = meta["steps"], meta["checkpoint"]
    prob = AD.FreeProblem(lat=lat, ps=ps, steps=T, window=K, storage=meta["storage"])
    F, tau = np.array(lat.body_force), lat.tau
    _, run = AD.forward_free(prob, F, tau, keep=True)   # allocations
    AD.backward_free(run)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J, run = AD.forward_free(prob, F, tau, keep=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    s0, dF, dtau = AD.backward_free(run)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    out = dict(steps=T, checkpoint=K, J=J, forward_steps_per_s=round(T / (t1 - t0), 1),
               adjoint_steps_per_s=round(T / (t2 - t1), 1),
               grad=dict(dJ_dx0=s0[0, 0:3].tolist(), dJ_dtheta0=s0[0, 3:6].tolist(),
                         dJ_dv0=s0[0, 6:9].tolist(), dJ_domega0=s0[0, 9:12].tolist(),
                         dJ_dF=dF.tolist(), dJ_dtau=dtau))
    print(f"[bench] free-motion adjoint: forward {t1 - t0:.2f} s, backward {t2 - t1:.2f} s",
          file=sys.stderr, flush=True)
    if fd_check:
        ref = dataclasses.replace(prob, storage="f64")

        def at(d):
            p2 = ps.copy()
            p2.vel = p2.vel.copy()
            p2.vel[0, 0] += d
            return AD.evaluate_free(dataclasses.replace(ref, ps=p2), F, tau)
        # steps small enough that no node changes owner between the runs (a
        # change of v0 by h moves the body by at most ~2000 h over the run);
        # two step sizes that agree show that none did
        fds = {}
        for h in (1e-8, 4e-8):
            fds[h] = (at(h) - at(-h)) / (2 * h)
        fd = fds[1e-8]
        out["fd_rel_err_v0x"] = float(abs(s0[0, 6] - fd) / abs(fd))
        out["fd_v0x"] = {f"h={h:g}": float(v) for h, v in fds.items()}
        out["fd_step_agreement"] = float(abs(fds[1e-8] - fds[4e-8]) / abs(fds[1e-8]))
        out["fd_reference"] = "central differences of the FP64-storage free-motion pass"
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c4", choices=["c2", "c3", "c4"])
    ap.add_argument("--storage", default="f32", choices=["f32", "f16", "f64"])
    ap.add_argument("--lattice", type=int, default=19, choices=[19, 15],
                    help="lattice of the timed line: D3Q19, or the paper's D3Q15")
    ap.add_argument("--variants", default="f16,f64,q15",
                    help="other storages timed on the same workload, and q15 for the "
                         "paper's D3Q15 lattice in the main storage (comma list, or none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-drag", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-fd", action="store_true",
                    help="skip the finite-difference checks of the adjoint gradients")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: --gpus {args.gpus} is not supported "
              "(the lattice update here runs on a single MI355X)", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a ROCm GPU", file=sys.stderr)
        sys.exit(2)
    from paper_2206_11634_amd import workloads as W

    lat, ps, meta = W.WORKLOADS[args.workload]()
    print(f"[bench] workload {meta['name']}: {lat.nx}x{lat.ny}x{lat.nz}, {ps.n} particles",
          file=sys.stderr, flush=True)
    main_res = run_storage(lat, ps, meta, args.storage, args.steps, args.warmup,
                           lattice=args.lattice, seq_steps=min(args.steps, 10))
    print(f"[bench] {args.storage}: {main_res['ms_per_step']:.3f} ms/step", file=sys.stderr,
          flush=True)
    variants, lattices = {}, {}
    for v in [s for s in args.variants.split(",") if s and s != "none" and s != args.storage]:
        if v == "q15" and args.lattice == 15:
            continue
        if v == "q15":
            r = run_storage(lat, ps, meta, args.storage, max(3, min(args.steps, 10)), 2,
                            lattice=15)
            lattices[f"d3q15_{args.storage}"] = r
        else:
            r = run_storage(lat, ps, meta, v, max(3, min(args.steps, 10)), 2)
            variants[v] = r
        print(f"[bench] {v}: {r['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)

    ncell = lat.ncell
    mlups = ncell / (main_res["ms_per_step"] * 1e-3) / 1e6
    nfluid = ncell - main_res["n_solid"]
    phases = {k: round(v[0] / max(v[1], 1), 4) for k, v in main_res["prof"].items() if v[1]}
    line = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_res["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.storage == "f64" else "f32",
        "data": "synthetic (seeded metaball suspension; no dataset)",
        "config": {
            "workload": meta["name"],
            "lattice": [lat.nx, lat.ny, lat.nz],
            "periodic": list(lat.periodic),
            "particles": ps.n,
            "storage": args.storage,
            "stencil": f"D3Q{args.lattice}",
            "tau": lat.tau,
            "treatments": int(meta.get("treatments", 3)),
            "dem_substeps": meta.get("n_sub", 10),
            "step": "classify + step with the dem sub-cycle beside its stream-collide pass + forces",
        },
        "fluid_mlups": round(nfluid / (main_res["ms_per_step"] * 1e-3) / 1e6, 1),
        "phase_ms_per_launch": phases,
        "links": main_res["n_links"],
        "link_candidates": main_res["n_cand"],
        "solid_fraction": round(main_res["n_solid"] / ncell, 4),
        "refills_last_step": main_res["n_refill"],
        "roofline": bulk_roofline(main_res, lat, args.storage, meta["name"], Q=args.lattice),
    }
    # context for the fraction: the same bytes moved by a plain copy
    ceil = copy_ceiling(args.lattice * lat.ncell * BYTES[args.storage])
    line["roofline"]["copy_ceiling"] = dict(achieved=ceil, unit="GB/s",
                                            frac_of_copy=round(line["roofline"]["achieved"] / ceil, 4))
    if main_res["seq"]:
        # the stream-collide pass with the chip to itself (lbm_step, then
        # dem_step), timed after the timed steps over a few more
        seq = dict(main_res, prof=main_res["seq"]["prof"])
        alone = bulk_roofline(seq, lat, args.storage, meta["name"], Q=args.lattice)
        line["roofline"]["alone"] = dict(avg_ms=alone["avg_ms"], achieved=alone["achieved"],
                                         frac=alone["frac"])
        line["sequential_ms_per_step"] = round(main_res["seq"]["ms_per_step"], 4)
    for v, r in variants.items():
        line.setdefault("storage_variants", {})[v] = dict(
            mlups=round(ncell / (r["ms_per_step"] * 1e-3) / 1e6, 1),
            ms_per_step=round(r["ms_per_step"], 4),
            roofline_frac=bulk_roofline(r, lat, v)["frac"])
    for v, r in lattices.items():
        rl = bulk_roofline(r, lat, args.storage, Q=15)
        line.setdefault("lattice_variants", {})[v] = dict(
            mlups=round(ncell / (r["ms_per_step"] * 1e-3) / 1e6, 1),
            ms_per_step=round(r["ms_per_step"], 4),
            phase_ms_per_launch={k: round(t[0] / max(t[1], 1), 4)
                                 for k, t in r["prof"].items() if t[1]},
            links=r["n_links"], roofline_achieved=rl["achieved"], roofline_frac=rl["frac"],
            bytes_per_cell=rl["bytes_per_cell"])
    if "f64" in variants:
        line["speedup_vs_plain_f64"] = round(variants["f64"]["ms_per_step"] /
                                             main_res["ms_per_step"], 3)
    if not args.no_drag:
        line["drag_err"] = drag_errors()
        line["exact_q"] = exact_q_effect(lat, ps, meta)
        c4 = line["drag_err"].get("c4", {})
        if "f64" in variants and "f32" in c4 and "f64" in c4:
            line["speedup_vs_plain_f64_equal_accuracy"] = dict(
                speedup=line["speedup_vs_plain_f64"],
                f32_within_bar=c4["f32"]["within_bar"], f64_within_bar=c4["f64"]["within_bar"])
    if not args.no_adjoint:
        line["adjoint"] = adjoint_bench(fd_check=not args.no_fd)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
