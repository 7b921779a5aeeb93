"""Gradient of a time-averaged hydrodynamic force (differentiation form).

J(v, F, tau) = sum over steps n < T of wF . F^h(n) + wT . T^h(n) for a run in
which the particles follow a prescribed rigid trajectory: their poses are
those of a nominal velocity v0 (so the geometry schedule -- owners, links, q,
refill sets -- is fixed), while the velocities the fluid sees (wall
velocities of bounce-back, refilling and momentum exchange) are v.  The
initial populations f(0) are data of the problem (by default the library's
initial equilibrium for the nominal F), not a function of (v, F, tau).  The
gradient with respect to v, the fluid body force F and the relaxation time
tau comes from the library's adjoint, run backwards window by window with
checkpoints every `window` steps and recomputation inside each window.

With geometry=True the adjoint also returns, for every pose of the
trajectory, dJ/dx_p (translation) and dJ/dtheta_p (small world-frame
rotation about x_p), with the link set, owners and refill sets held fixed
(q, the wall points and the lever arms move with the body).  From them follow
the derivatives with respect to the initial pose and the full derivative
with respect to a velocity that drives both the poses and the wall
velocities (`trajectory_gradients`).

`DragFunction` wraps this as a torch.autograd.Function of (v, F, tau).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import binding as B
from . import workloads as W


@dataclasses.dataclass
class Problem:
    lat: W.LatticeSpec
    ps: W.ParticleSet          # initial state; ps.vel is the nominal velocity v0
    steps: int
    window: int = 100
    storage: str = "f32"
    weights: np.ndarray = None  # [n][6]: (wF, wT) per particle per step
    f0: np.ndarray = None       # [Q][ncell] initial populations
    treatments: int = B.TREAT_VIBB | B.TREAT_MISSING
    lattice: int = 19           # 19 (D3Q19) or 15 (D3Q15)
    keep_geometry: bool = True  # keep every step's geometry for the replay (about
                                # owner_bytes + flag_bytes per step on the device)

    def __post_init__(self):
        if self.weights is None:
            w = np.zeros((self.ps.n, 6))
            w[0, 0] = 1.0 / self.steps    # mean x-force on particle 0
            self.weights = w

    def states(self):
        """Nominal particle states at steps 0..T (poses of the prescribed
        trajectory; the geometry schedule)."""
        if getattr(self, "_states", None) is None:
            self._states = [W.prescribed_state(self.ps, self.lat, float(n))
                            for n in range(self.steps + 1)]
        return self._states

    def initial(self) -> np.ndarray:
        if self.f0 is None:
            g = B.Lattice.for_particles(self.lat, self.ps, storage="f64", lattice=self.lattice)
            self.f0 = g.populations()
            g.close()
        return self.f0


class _Run:
    def __init__(self, prob: Problem, vel, body_force, tau):
        self.prob = prob
        self.vel = np.asarray(vel, float).reshape(prob.ps.n, 3)
        self.lat = dataclasses.replace(prob.lat, body_force=tuple(map(float, body_force)),
                                       tau=float(tau))
        self.gpu = B.Lattice.for_particles(self.lat, prob.ps, storage=prob.storage,
                                           treatments=prob.treatments, lattice=prob.lattice)
        # every state on the device: poses of the nominal trajectory, velocity v
        self.traj = B.DeviceTrajectory(prob.states(), vel=self.vel)
        self.second = self.stream2 = None

    def parts(self, n):
        return self.traj[n]

    def open_second(self):
        """A second lattice context on a stream of its own (default
        priority), which replays the windows of the backward pass beside the
        adjoint of the window after them; its lists are sized by the
        classification at the first pose, as the forward pass's were."""
        torch = self.gpu.torch
        self.stream2 = torch.cuda.Stream(device=self.gpu.device)
        with torch.cuda.stream(self.stream2):
            self.second = B.Lattice.for_particles(self.lat, self.prob.ps,
                                                  storage=self.prob.storage,
                                                  treatments=self.prob.treatments,
                                                  lattice=self.prob.lattice)
            self.second.classify(self.parts(0))

    def close(self):
        if self.second is not None:
            self.second.close()
            self.second = None
        self.gpu.close()


def _again_with_read_back(fn):
    """Run fn(sync=False) -- classifications without the host read-back --
    and, should a list outgrow its capacity there (reported at the end of the
    run), run fn(sync=True), whose classifications grow the lists."""
    try:
        return fn(sync=False)
    except B.LbmError as e:
        if e.code != B.LBM_ECAPACITY:
            raise
    return fn(sync=True)


def _snapshot(run, k):
    """Keep the geometry of the classification just made as that of step k."""
    if run.prob.keep_geometry:
        run.geo[k] = run.gpu.geometry_save()


def _second_fits(run) -> bool:
    """Whether the device has room for a second context and its tape beside
    the first context's tape: a window's populations and owner planes, twice,
    and the second context's own buffers, with a quarter to spare."""
    gpu = run.gpu
    z = gpu.sizes
    tape = run.prob.window * (z.population_bytes + z.owner_bytes + (1 << 20))
    ctx = 2 * z.population_bytes + 2 * z.owner_bytes + z.flag_bytes + z.moment_bytes
    free, _ = gpu.torch.cuda.mem_get_info(gpu.device)
    return free > 1.25 * (2 * tape + ctx)


def _replay_classify(run, k, parts, gpu=None):
    """In a replay: the forward pass's geometry of step k if it kept one that
    fits the list capacities of now, else a classification (asynchronous:
    the forward pass sized the lists for the same poses)."""
    gpu = run.gpu if gpu is None else gpu
    snap = run.geo.get(k)
    if snap is not None and snap[1] == gpu.geometry_bytes()[1]:
        gpu.geometry_load(snap, parts)
    else:
        gpu.classify(parts, sync=False)


def _replay(run, gpu, w0, w1):
    """Restore the checkpoint of step w0 on gpu and run steps w0 .. w1 - 1
    again with the tape on (asynchronous, on gpu's stream)."""
    gpu.restore(run.ckpt[w0])
    # the geometry of the forward pass, or classifications without
    # read-backs (lbm_adjoint reports anything they latched)
    _replay_classify(run, w0, run.parts(w0), gpu)   # the geometry at w0, refills nothing
    gpu.tape_begin(w1 - w0)
    for k in range(w0, w1):
        gpu.step(run.parts(k))
        _replay_classify(run, k + 1, run.parts(k + 1), gpu)


def _closing(gpu, body):
    try:
        return body()
    except BaseException:
        gpu.close()
        raise


def forward(prob: Problem, vel, body_force, tau, keep: bool = False):
    """Run the forward pass; J, and the run (with its checkpoints) if keep."""
    return _again_with_read_back(
        lambda sync: _forward(prob, vel, body_force, tau, keep, sync))


def _forward(prob: Problem, vel, body_force, tau, keep: bool, sync: bool):
    run = _Run(prob, vel, body_force, tau)
    gpu, T, n = run.gpu, prob.steps, prob.ps.n
    torch = gpu.torch

    def body():
        gpu.set_populations(prob.initial())
        run.ckpt, run.geo = {}, {}
        hist = torch.zeros((T, 2, max(n, 1), 3), dtype=torch.float64, device=gpu.device)
        gpu.classify(run.parts(0))   # sizes the lists
        if keep:
            _snapshot(run, 0)
        for k in range(T):
            if keep and k % prob.window == 0:
                run.ckpt[k] = gpu.checkpoint()
            gpu.step(run.parts(k))
            gpu.forces(hist[k, 0], hist[k, 1])
            gpu.classify(run.parts(k + 1), sync=sync)
            if keep:
                _snapshot(run, k + 1)
        gpu.sync()   # reports what the classifications latched
        w = torch.as_tensor(prob.weights, dtype=torch.float64, device=gpu.device)
        return float((hist[:, 0, :n] * w[:, :3]).sum() + (hist[:, 1, :n] * w[:, 3:]).sum())

    J = _closing(gpu, body)
    if not keep:
        gpu.close()
        return J, None
    return J, run


def backward(run: _Run, stats: dict | None = None, geometry: bool = False):
    """(dJ/dv [n][3], dJ/dF [3], dJ/dtau) by the adjoint, window by window from
    the last checkpoint to the first, recomputing each window's steps; with
    geometry, also (dJ/dx_p, dJ/dtheta_p) of every pose [T + 1][n][6].  With
    a dict for stats, the library's per-phase timers are read into it."""
    prob, gpu = run.prob, run.gpu
    torch = gpu.torch
    wins = sorted(run.ckpt, reverse=True)
    # With the forward pass's geometry kept, window i's replay runs on a
    # second context (its own stream), beside the adjoint of window i - 1 on
    # the first, alternating; an adjoint call waits for its own stream only,
    # and the adjoint field and the sums pass from one adjoint call to the
    # next after the host has waited for the first.  The second context must
    # load the same snapshots (the same list capacities) and its tape must
    # fit beside the first's; otherwise one context replays and runs the
    # adjoint of each window in turn.
    two = len(wins) > 1 and prob.keep_geometry and (run.second is not None or _second_fits(run))
    if two and run.second is None:
        run.open_second()
    if two and run.second.geometry_bytes()[1] != gpu.geometry_bytes()[1]:
        run.second.close()
        run.second, two = None, False
    ctxs = [gpu, run.second] if two else [gpu]
    streams = [torch.cuda.current_stream(gpu.device), run.stream2]
    if stats is not None:
        for c in ctxs:
            c.profile(True)
    lam = gpu.adjoint_field()
    n = prob.ps.n
    g = torch.zeros(4 + 3 * n, dtype=torch.float64, device=gpu.device)
    gx = (torch.zeros((prob.steps + 1, max(n, 1), 6), dtype=torch.float64, device=gpu.device)
          if geometry else None)
    torch.cuda.synchronize(gpu.device)   # lam, g and gx are set before either stream reads them

    def span(w0):
        return w0, min(w0 + prob.window, prob.steps)

    def adjoint(c, w0):
        w1 = span(w0)[1]
        # poses w0 .. w1 of this window: a contiguous view of gx
        c.adjoint(run.parts(w1), prob.weights, lam, g, None if gx is None else gx[w0:w1 + 1])

    try:
        if two:
            with torch.cuda.stream(streams[0]):
                _replay(run, ctxs[0], *span(wins[0]))
            for i, w0 in enumerate(wins):
                if i + 1 < len(wins):
                    with torch.cuda.stream(streams[(i + 1) % 2]):
                        _replay(run, ctxs[(i + 1) % 2], *span(wins[i + 1]))
                with torch.cuda.stream(streams[i % 2]):
                    adjoint(ctxs[i % 2], w0)
        else:
            for w0 in wins:
                _replay(run, gpu, *span(w0))
                adjoint(gpu, w0)
        torch.cuda.synchronize(gpu.device)
        out = g.cpu().numpy()
        if stats is not None:
            for c in ctxs:
                for k, (ms, cnt) in c.profile_read().items():
                    a = stats.get(k, (0.0, 0))
                    stats[k] = (a[0] + ms, a[1] + cnt)
                c.profile(False)
    finally:
        run.close()   # waits for both streams
    res = (out[4:].reshape(n, 3), out[:3].copy(), float(out[3]))
    if geometry:
        res = res + (gx[:, :n].cpu().numpy(),)
    return res


def evaluate(prob: Problem, vel, body_force, tau, grad: bool = False, geometry: bool = False):
    """J, and with grad=True also (dJ/dv [n][3], dJ/dF [3], dJ/dtau), and with
    geometry=True also (dJ/dx_p, dJ/dtheta_p) of every pose [T + 1][n][6]."""
    J, run = forward(prob, vel, body_force, tau, keep=grad)
    if not grad:
        return J
    return (J,) + backward(run, geometry=geometry)


def trajectory_gradients(prob: Problem, gx: np.ndarray, dv: np.ndarray):
    """For the prescribed trajectory x_p(k) = x_p(0) + v0 k,
    q_p(k) = exp(omega k / 2) q_p(0):
      dJ/dx_p(0)     = sum_k dJ/dx_p(k);
      dJ/dv0         = dJ/dv + sum_k k dJ/dx_p(k), v0 driving both the poses
                       and the wall velocities;
      dJ/dtheta_p(0) = sum_k R_k^T dJ/dtheta_p(k) for a small world-frame
                       rotation of the initial orientation, which reaches
                       pose k rotated by R_k = R(exp(omega k / 2))."""
    T1, n = gx.shape[0], gx.shape[1]
    k = np.arange(T1, dtype=float)[:, None, None]
    gt0 = np.zeros((n, 3))
    for p in range(n):
        w = prob.ps.omega[p]
        wn = float(np.linalg.norm(w))
        for j in range(T1):
            if wn > 0:
                a = 0.5 * wn * j
                R = W.quat_to_matrix(np.concatenate([[np.cos(a)], np.sin(a) * w / wn]))
            else:
                R = np.eye(3)
            gt0[p] += R.T @ gx[j, p, 3:]
    return gx[:, :, :3].sum(0), dv + (k * gx[:, :, :3]).sum(0), gt0


# ---------------------------------------------------------------------------
# free motion: the particles follow the DEM under the step's forces
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class FreeProblem:
    """J(s_0) = sum over steps k < T of wF . F^h(k) + wT . T^h(k) for a run in
    which, after every lattice step, dem_step advances the particles (n_sub
    substeps of 1/n_sub) under F^h, T^h and relative gravity.  The gradient
    is with respect to the initial state s_0 = (x, theta, v, omega) of every
    particle (theta a small world-frame rotation of the initial orientation),
    the fluid body force and tau, through the DEM's contact forces as well
    (contact clusters of at most 8 particles per dem_step call)."""
    lat: W.LatticeSpec
    ps: W.ParticleSet
    steps: int
    window: int = 100
    storage: str = "f32"
    weights: np.ndarray = None
    f0: np.ndarray = None
    treatments: int = B.TREAT_VIBB | B.TREAT_MISSING
    lattice: int = 19
    gravity: tuple = (0.0, 0.0, 0.0)
    n_sub: int = 10
    keep_geometry: bool = True

    def __post_init__(self):
        if self.weights is None:
            w = np.zeros((self.ps.n, 6))
            w[0, 0] = 1.0 / self.steps
            self.weights = w

    def dem(self):
        return B.DemParams.make(**W.dem_defaults(self.ps, gravity=self.gravity))


class _FreeRun:
    def __init__(self, prob: FreeProblem, body_force, tau):
        self.prob = prob
        self.lat = dataclasses.replace(prob.lat, body_force=tuple(map(float, body_force)),
                                       tau=float(tau))
        self.gpu = B.Lattice.for_particles(self.lat, prob.ps, storage=prob.storage,
                                           treatments=prob.treatments, lattice=prob.lattice)
        self.parts = B.DeviceParticles(prob.ps)
        self.prm = prob.dem()
        self.dt = 1.0 / prob.n_sub
        self.second = self.parts2 = self.stream2 = None

    def state(self):
        """The particle arrays and the DEM's own state (contact histories and
        the carried contact sums), which a replayed window starts from."""
        st = {k: self.parts.t[k].clone() for k in ("pos", "quat", "vel", "omega", "world_pts")}
        st["dem"] = self.gpu.dem_checkpoint()
        return st

    def load(self, st, gpu=None, parts=None):
        gpu = self.gpu if gpu is None else gpu
        parts = self.parts if parts is None else parts
        for k, v in st.items():
            if k == "dem":
                gpu.dem_restore(v)
            else:
                parts.t[k].copy_(v)

    def advance(self, sync: bool = True, replay_step: int | None = None, gpu=None, parts=None):
        """dem_step, then the classification of the new poses (in a replay,
        step replay_step's geometry kept by the forward pass, if any)."""
        gpu = self.gpu if gpu is None else gpu
        parts = self.parts if parts is None else parts
        gpu.dem(parts, self.prob.n_sub, self.dt, self.prm)
        if replay_step is None:
            gpu.classify(parts, sync=sync)
        else:
            _replay_classify(self, replay_step, parts, gpu)

    def open_second(self):
        """A second lattice context with particle arrays of its own, on a
        stream of its own (default priority), for the replays of the backward
        pass; its lists are sized at the initial state, as the forward pass's
        were."""
        torch = self.gpu.torch
        self.stream2 = torch.cuda.Stream(device=self.gpu.device)
        with torch.cuda.stream(self.stream2):
            self.second = B.Lattice.for_particles(self.lat, self.prob.ps,
                                                  storage=self.prob.storage,
                                                  treatments=self.prob.treatments,
                                                  lattice=self.prob.lattice)
            self.parts2 = B.DeviceParticles(self.prob.ps)
            self.second.classify(self.parts2)

    def close(self):
        if self.second is not None:
            self.second.close()
            self.second = None
        self.gpu.close()


def forward_free(prob: FreeProblem, body_force, tau, keep: bool = False):
    """J of the free-motion run, and the run (with checkpoints of the lattice,
    of the particle state and of the DEM state at every window start) if
    keep."""
    return _again_with_read_back(lambda sync: _forward_free(prob, body_force, tau, keep, sync))


def _forward_free(prob: FreeProblem, body_force, tau, keep: bool, sync: bool):
    run = _FreeRun(prob, body_force, tau)
    gpu, T, n = run.gpu, prob.steps, prob.ps.n
    torch = gpu.torch

    def body():
        if prob.f0 is not None:
            gpu.set_populations(prob.f0)
        run.ckpt, run.geo = {}, {}
        hist = torch.zeros((T, 2, max(n, 1), 3), dtype=torch.float64, device=gpu.device)
        gpu.classify(run.parts)   # sizes the lists
        if keep:
            _snapshot(run, 0)
        for k in range(T):
            if keep and k % prob.window == 0:
                run.ckpt[k] = (gpu.checkpoint(), run.state())
            gpu.step(run.parts)
            gpu.forces(hist[k, 0], hist[k, 1])
            run.advance(sync)
            if keep:
                _snapshot(run, k + 1)
        gpu.sync()   # reports what the classifications latched
        w = torch.as_tensor(prob.weights, dtype=torch.float64, device=gpu.device)
        return float((hist[:, 0, :n] * w[:, :3]).sum() + (hist[:, 1, :n] * w[:, 3:]).sum())

    J = _closing(gpu, body)
    if not keep:
        gpu.close()
        return J, None
    return J, run


def backward_free(run: _FreeRun):
    """(dJ/ds_0 [n][12] ordered x, theta, v, omega; dJ/dF [3]; dJ/dtau) by the
    coupled adjoint, window by window from the last checkpoint."""
    prob, gpu = run.prob, run.gpu
    torch = gpu.torch
    n = prob.ps.n
    wins = sorted(run.ckpt, reverse=True)
    # as in backward: with the forward pass's geometry kept, a second context
    # (particle arrays and stream of its own) replays window i beside the
    # adjoint of window i - 1, alternating
    two = len(wins) > 1 and prob.keep_geometry and (run.second is not None or _second_fits(run))
    if two and run.second is None:
        run.open_second()
    if two and run.second.geometry_bytes()[1] != gpu.geometry_bytes()[1]:
        run.second.close()
        run.second, two = None, False
    lanes = [(gpu, run.parts), (run.second, run.parts2)] if two else [(gpu, run.parts)]
    streams = [torch.cuda.current_stream(gpu.device), run.stream2]
    lam = gpu.adjoint_field()
    g = torch.zeros(4, dtype=torch.float64, device=gpu.device)
    sig = torch.zeros((max(n, 1), 12), dtype=torch.float64, device=gpu.device)
    sigc = gpu.contact_adjoint()   # carried contact sums and springs, across windows
    torch.cuda.synchronize(gpu.device)   # set before either stream reads them

    def replay(lane, w0):
        c, parts = lane
        w1 = min(w0 + prob.window, prob.steps)
        ck, st = run.ckpt[w0]
        c.restore(ck)
        run.load(st, c, parts)
        # replayed poses: the forward pass's geometry, or classifications
        # without read-backs (lbm_adjoint_coupled reports anything they latched)
        _replay_classify(run, w0, parts, c)   # the geometry at w0, refills nothing
        c.tape_begin(w1 - w0)
        for k in range(w0, w1):
            c.step(parts)
            run.advance(replay_step=k + 1, gpu=c, parts=parts)

    def adjoint(lane):
        c, parts = lane
        c.adjoint_coupled(parts, prob.weights, run.prm, prob.n_sub, run.dt, lam, g, sig, sigc)

    try:
        if two:
            with torch.cuda.stream(streams[0]):
                replay(lanes[0], wins[0])
            for i in range(len(wins)):
                if i + 1 < len(wins):
                    with torch.cuda.stream(streams[(i + 1) % 2]):
                        replay(lanes[(i + 1) % 2], wins[i + 1])
                with torch.cuda.stream(streams[i % 2]):
                    adjoint(lanes[i % 2])
        else:
            for w0 in wins:
                replay(lanes[0], w0)
                adjoint(lanes[0])
        torch.cuda.synchronize(gpu.device)
        out = g.cpu().numpy()
        s0 = sig[:n].cpu().numpy()
    finally:
        run.close()   # waits for both streams
    return s0, out[:3].copy(), float(out[3])


def evaluate_free(prob: FreeProblem, body_force, tau, grad: bool = False):
    """J, and with grad=True also (dJ/ds_0 [n][12], dJ/dF [3], dJ/dtau)."""
    J, run = forward_free(prob, body_force, tau, keep=grad)
    if not grad:
        return J
    return (J,) + backward_free(run)


def _make_function():
    import torch

    class DragFunction(torch.autograd.Function):
        """J = DragFunction.apply(v [n,3], F [3], tau [], problem): the forward
        pass keeps checkpoints; the backward pass runs the adjoint."""

        @staticmethod
        def forward(ctx, vel, body_force, tau, prob):
            J, run = forward(prob, vel.detach().cpu().numpy(), body_force.detach().cpu().numpy(),
                             float(tau.detach().cpu()), keep=True)
            ctx.run = run
            return torch.tensor(J, dtype=torch.float64)

        @staticmethod
        def backward(ctx, gJ):
            dv, dF, dtau = backward(ctx.run)
            ctx.run = None
            return (gJ * torch.as_tensor(dv), gJ * torch.as_tensor(dF),
                    gJ * torch.as_tensor(dtau), None)

    return DragFunction


def __getattr__(name):
    if name == "DragFunction":
        return _make_function()
    raise AttributeError(name)


def main(argv=None):
    """Forward and adjoint of the 128^3 channel with one metaball at a
    prescribed velocity (FP32 storage, 2000 steps, checkpoints every 100):
    steps per second of each pass and the gradient, as one JSON line."""
    import argparse
    import json
    import sys
    import time

    import torch

    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--steps", type=int, default=None, help="steps (default: the workload's 2000)")
    ap.add_argument("--repeat", type=int, default=1, help="forward + adjoint passes to time")
    args = ap.parse_args(argv)
    if not torch.cuda.is_available():
        print("the adjoint runs on a ROCm GPU", file=sys.stderr)
        return 2
    lat, ps, meta = W.config_c5()
    T = args.steps or meta["steps"]
    prob = Problem(lat=lat, ps=ps, steps=T, window=meta["checkpoint"], storage=meta["storage"])
    v, F, tau = ps.vel.copy(), np.array(lat.body_force), lat.tau
    prob.initial()
    for _ in range(args.repeat):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        J, run = forward(prob, v, F, tau, keep=True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        dv, dF, dtau = backward(run)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        print(json.dumps(dict(workload=meta["name"], steps=T, J=J,
                              forward_steps_per_s=round(T / (t1 - t0), 1),
                              adjoint_steps_per_s=round(T / (t2 - t1), 1),
                              dJ_dU=dv[0].tolist(), dJ_dF=dF.tolist(), dJ_dtau=dtau)),
              flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
