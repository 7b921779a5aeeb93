"""Pins of the oracle's bulk lattice update (Sec. 2.2) against closed forms
and invariants that do not come from the oracle itself."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2206_11634_amd import workloads as W


def _empty():
    return W.make_particles([], np.zeros((0, 3)), np.zeros((0, 4)), 1.0)


@pytest.mark.parametrize("Q", [19, 15])
def test_stencil_isotropy(Q):
    """Weights reproduce the Maxwellian moments up to fourth order with c_s^2 = 1/3."""
    e, w, opp = O.stencil(Q)
    e = e.astype(float)
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.abs((w[:, None] * e).sum(0)).max() < 1e-16
    M2 = np.einsum("i,ia,ib->ab", w, e, e)
    assert np.allclose(M2, np.eye(3) / 3.0, atol=1e-16)
    M4 = np.einsum("i,ia,ib,ic,id->abcd", w, e, e, e, e)
    d = np.eye(3)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
           + np.einsum("ad,bc->abcd", d, d)) / 9.0
    assert np.allclose(M4, iso, atol=1e-16)
    assert np.all(e[opp] == -e)
    if Q == 19:  # the exported numbering: opposite of odd i is i + 1
        assert all(opp[i] == i + 1 for i in range(1, 19, 2))


def test_rest_state_with_particles_and_walls():
    """Fluid at rest around particles at rest stays at f = w (to rounding)."""
    lat, ps = W.tiny_case(11, dims=(18, 16, 14), periodic=(1, 0, 0), n_particles=3)
    o = O.Oracle(lat)
    o.classify(ps)
    _, w, _ = O.stencil(19)
    for _ in range(20):
        F, T = o.step(ps)
        o.classify(ps)
    fl = o.owner == 0
    assert np.abs(o.f[:, fl] - w[:, None]).max() < 1e-15
    assert np.abs(F).max() < 1e-13 and np.abs(T).max() < 1e-12


@pytest.mark.parametrize("per", [(1, 1, 1), (1, 0, 1), (0, 0, 0)])
def test_mass_conservation_without_particles(per):
    """Streaming, BGK collision and halfway walls conserve sum f exactly (to rounding)."""
    rng = np.random.default_rng(3)
    lat = W.LatticeSpec(12, 10, 8, per, tau=0.63)
    o = O.Oracle(lat)
    o.classify(_empty())
    o.f *= 1.0 + 0.01 * rng.standard_normal(o.f.shape)
    m0 = o.f.sum()
    for _ in range(40):
        o.step(_empty())
    assert abs(o.f.sum() - m0) / m0 < 1e-13


def test_poiseuille_exact_at_magic_tau():
    """BGK + Guo forcing + halfway walls give the parabola
    u(y) = g/(2 nu) (y + 1/2)(H - 1/2 - y) exactly when (tau - 1/2)^2 = 3/16."""
    tau = 0.5 + np.sqrt(3.0) / 4.0
    H, g = 8, 1e-6
    lat = W.LatticeSpec(3, H, 3, (1, 0, 1), tau=tau, body_force=(g, 0, 0))
    o = O.Oracle(lat)
    o.classify(_empty())
    nu = (tau - 0.5) / 3.0
    for _ in range(int(20 * H * H / nu)):
        o.step(_empty())
    _, u = o.moments()
    ux = o.field(u[:, 0])[1, :, 1]
    y = np.arange(H)
    ua = g / (2 * nu) * (y + 0.5) * (H - 0.5 - y)
    assert np.abs(ux - ua).max() / ua.max() < 1e-9
    assert np.abs(u[:, 1:]).max() < 1e-10 * ua.max()


def test_poiseuille_second_order_off_magic_tau():
    tau, g = 0.8, 1e-6
    errs = []
    for H in (8, 16):
        lat = W.LatticeSpec(3, H, 3, (1, 0, 1), tau=tau, body_force=(g, 0, 0))
        o = O.Oracle(lat)
        o.classify(_empty())
        nu = (tau - 0.5) / 3.0
        for _ in range(int(12 * H * H / nu)):
            o.step(_empty())
        _, u = o.moments()
        ux = o.field(u[:, 0])[1, :, 1]
        y = np.arange(H)
        ua = g / (2 * nu) * (y + 0.5) * (H - 0.5 - y)
        errs.append(np.abs(ux - ua).max() / ua.max())
    order = np.log2(errs[0] / errs[1])
    assert 1.8 < order < 2.2, (errs, order)


def _shear_wave_rate_error(L, tau=0.7, U=1e-4):
    lat = W.LatticeSpec(2, L, 2, (1, 1, 1), tau=tau)
    o = O.Oracle(lat)
    o.classify(_empty())
    e, w, _ = O.stencil(19)
    y = np.arange(L)
    uf = np.broadcast_to((U * np.sin(2 * np.pi * y / L))[None, :, None], (2, L, 2)).reshape(-1)
    eu = e[:, 0][:, None] * uf[None, :]
    o.f = np.ascontiguousarray(w[:, None] * (1 + 3 * eu + 4.5 * eu ** 2 - 1.5 * uf[None, :] ** 2))
    nu = (tau - 0.5) / 3.0
    k = 2 * np.pi / L
    nsteps = int(1.5 / (nu * k * k))
    amps = []
    for _ in range(nsteps):
        o.step(_empty())
        _, u = o.moments()
        amps.append(abs(o.field(u[:, 0])[0, :, 0] @ np.sin(2 * np.pi * y / L)) * 2 / L)
    t = np.arange(1, nsteps + 1)
    h = nsteps // 4
    rate = -np.polyfit(t[h:], np.log(np.array(amps[h:])), 1)[0]
    return abs(rate / (nu * k * k) - 1.0)


def test_shear_wave_viscous_decay():
    """u_x = U sin(2 pi y / L) decays as exp(-nu k^2 t) with nu = (tau - 1/2)/3,
    up to the lattice's O(k^2) dispersion, which must shrink fourfold when L doubles."""
    e32 = _shear_wave_rate_error(32)
    e64 = _shear_wave_rate_error(64)
    assert e32 < 4e-3 and e64 < 1e-3
    assert 3.0 < e32 / e64 < 5.0, (e32, e64)


def test_uniform_body_force_momentum():
    """With a uniform force density F, the n-th collision uses u = (n - 1/2) F / rho
    and leaves momentum n F per node (Guo's half-force shift)."""
    Fv = np.array([2e-6, -1e-6, 5e-7])
    lat = W.LatticeSpec(4, 4, 4, (1, 1, 1), tau=0.9, body_force=tuple(Fv))
    o = O.Oracle(lat)
    o.classify(_empty())
    e, _, _ = O.stencil(19)
    for n in range(1, 11):
        o.step(_empty())
        rho, u = o.moments()
        mom = (o.f.T @ e.astype(float))
        assert np.allclose(mom, n * Fv[None, :], rtol=1e-9, atol=2e-15)
        assert np.allclose(u * rho[:, None], (n - 0.5) * Fv[None, :], rtol=1e-9, atol=2e-15)


def test_d3q15_runs_poiseuille():
    """The paper's D3Q15 lattice goes through the same generic code."""
    tau = 0.5 + np.sqrt(3.0) / 4.0
    H, g = 6, 1e-6
    lat = W.LatticeSpec(3, H, 3, (1, 0, 1), tau=tau, body_force=(g, 0, 0))
    o = O.Oracle(lat, Q=15)
    o.classify(_empty())
    nu = (tau - 0.5) / 3.0
    for _ in range(int(20 * H * H / nu)):
        o.step(_empty())
    rho, u = o.moments()
    ux = o.field(u[:, 0])[1, :, 1]
    y = np.arange(H)
    ua = g / (2 * nu) * (y + 0.5) * (H - 0.5 - y)
    assert np.abs(ux - ua).max() / ua.max() < 1e-8
