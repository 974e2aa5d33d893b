"""Pins of the scheme variants Sec. 3.2 describes, in the oracle (no GPU):
unsplit PLM with the reference state, the linearised approximate Riemann
solver, and the second form of the energy gravity term (the update of E is
the update of the kinetic energy)."""
import math

import numpy as np
import pytest

import oracle
from exact_riemann import sample
from paper_1301_4498_amd import synth

NG = 4
G = 5.0 / 3.0
PLM = oracle.Params(recon=oracle.RECON_PLM)
LIN = oracle.Params(riemann=oracle.RIEMANN_LINEAR)
GF2 = oracle.Params(grav_form=2)


def _valid(f):
    return f[:, NG:-NG, NG:-NG, NG:-NG]


# ---------------------------------------------------------------- PLM ----

def test_plm_edges_exact_on_linear_data_and_flattened():
    q = 0.3 + 0.7 * np.arange(12, dtype=float)
    qm, qp = oracle.plm_line(q)
    j = np.arange(2, 9)
    assert np.allclose(qm[j], q[j] - 0.35, rtol=0, atol=1e-14)
    assert np.allclose(qp[j], q[j] + 0.35, rtol=0, atol=1e-14)
    qm0, qp0 = oracle.plm_line(q, chi=np.zeros(12))
    assert np.array_equal(qm0[j], q[j]) and np.array_equal(qp0[j], q[j])
    half = np.full(12, 0.5)
    qmh, qph = oracle.plm_line(q, chi=half)
    assert np.allclose(qph[j] - q[j], 0.175, atol=1e-14)


def test_plm_edges_create_no_new_extrema():
    rng = np.random.default_rng(5)
    q = np.cumsum(rng.normal(size=64)) + rng.normal(size=64) * 3
    qm, qp = oracle.plm_line(q)
    for j in range(2, 61):
        lo, hi = min(q[j - 1:j + 2]), max(q[j - 1:j + 2])
        for e in (qm[j], qp[j]):
            assert lo - 1e-12 <= e <= hi + 1e-12, (j, e, lo, hi)


def test_plm_step_conserves_and_differs_from_ppm():
    w = synth.config1(n=16, seed=21)
    g = np.zeros_like(w.grav)
    dt = oracle.estimate_dt(w.state, NG, w.a0, w.dx, 0.5)
    out, st = oracle.hydro_step(w.state, g, NG, dt, w.dx, w.a0, w.a0 * 1.01, PLM)
    ppm, _ = oracle.hydro_step(w.state, g, NG, dt, w.dx, w.a0, w.a0 * 1.01)
    assert st["sync_E_from_e"] == 0
    v0, v1 = _valid(w.state), _valid(out)
    for c in range(5):
        s0, s1 = math.fsum(v0[c].ravel()), math.fsum(v1[c].ravel())
        assert abs(s1 - s0) <= 1e-13 * math.fsum(np.abs(v0[c]).ravel()), c
    assert not np.array_equal(_valid(ppm), v1)
    # a uniform state is preserved
    shape = (6, 6, 6)
    U = synth.pad_periodic(synth.conserved(np.full(shape, 1.3), np.stack(
        [np.full(shape, x) for x in (0.4, -0.7, 0.2)]), np.full(shape, 0.9), 0.7))
    o, _ = oracle.hydro_step(U, np.zeros((3,) + U.shape[1:]), NG, 0.01, 0.1, 0.7, 0.7, PLM)
    assert np.allclose(_valid(o), _valid(U), rtol=1e-13, atol=0)


def _entropy_wave_error(N, prm, U0=1.0, t_end=0.25):
    x = (np.arange(N) + 0.5) / N
    shape = (2, 2, N)

    def rho_avg(xc, t):
        h = 1.0 / N
        return 1.0 + 0.2 * (np.cos(2 * np.pi * (xc - h / 2 - U0 * t)) -
                            np.cos(2 * np.pi * (xc + h / 2 - U0 * t))) / (2 * np.pi * h)

    rho = np.broadcast_to(rho_avg(x, 0.0), shape).copy()
    u = np.stack([np.full(shape, U0), np.zeros(shape), np.zeros(shape)])
    U = synth.pad_periodic(synth.conserved(rho, u, np.ones(shape), 1.0))
    g = np.zeros((3,) + U.shape[1:])
    t = 0.0
    while t < t_end - 1e-14:
        dt = min(oracle.estimate_dt(U, NG, 1.0, 1.0 / N, 0.5, prm), t_end - t)
        U, _ = oracle.hydro_step(U, g, NG, dt, 1.0 / N, 1.0, 1.0, prm)
        synth.fill_periodic_inplace(U)
        t += dt
    return np.abs(_valid(U)[0][0, 0] - rho_avg(x, t_end)).mean()


def test_plm_entropy_wave_converges_at_second_order():
    errs = [_entropy_wave_error(N, PLM) for N in (32, 64, 128)]
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    ppm = _entropy_wave_error(64, oracle.Params())
    assert min(orders) >= 1.6, (errs, orders)
    assert errs[1] > ppm  # the parabola is the more accurate profile


# --------------------------------------------------- linearised solver ----

def test_linear_solver_is_exact_for_a_contact():
    qL = np.array([2.0, 0.3, 0.1, -0.2, 0.7])
    qR = np.array([0.5, 0.3, -0.4, 0.6, 0.7])
    for u in (0.3, -0.3):
        qL[1] = qR[1] = u
        qg, st, it = oracle.riemann(qL, qR, LIN)
        assert it == 0
        assert st["p"] == pytest.approx(0.7, rel=1e-15)
        assert st["u"] == pytest.approx(u, rel=1e-15)
        assert st["rhoL"] == pytest.approx(2.0, rel=1e-15)
        assert st["rhoR"] == pytest.approx(0.5, rel=1e-15)
        up = qL if u > 0 else qR
        assert np.allclose(qg, up, rtol=1e-14)


def test_linear_solver_agrees_with_two_shock_to_second_order():
    # weak waves: the linearised star state differs from the two-shock one by
    # O(amplitude^2); halving the jump quarters the difference
    base = np.array([1.0, 0.0, 0.0, 0.0, 1.0])
    dq = np.array([0.3, -0.5, 0.0, 0.0, 0.4])
    diffs = []
    for eps in (0.04, 0.02, 0.01):
        qL, qR = base + eps * dq, base - eps * dq
        _, sl, _ = oracle.riemann(qL, qR, LIN)
        _, st, _ = oracle.riemann(qL, qR)
        diffs.append(max(abs(sl["p"] - st["p"]), abs(sl["u"] - st["u"]),
                         abs(sl["rhoL"] - st["rhoL"]), abs(sl["rhoR"] - st["rhoR"])))
    r = [diffs[i] / diffs[i + 1] for i in range(2)]
    assert all(3.5 < x < 4.5 for x in r), (diffs, r)


def test_linear_solver_mirror_symmetry_and_floor():
    qL = np.array([1.2, 0.4, 0.1, 0.2, 0.9])
    qR = np.array([0.6, -0.3, 0.3, -0.1, 0.4])
    qg, st, _ = oracle.riemann(qL, qR, LIN)
    mL = qR * np.array([1, -1, 1, 1, 1])
    mR = qL * np.array([1, -1, 1, 1, 1])
    qg2, st2, _ = oracle.riemann(mL, mR, LIN)
    assert st2["p"] == pytest.approx(st["p"], rel=1e-14)
    assert st2["u"] == pytest.approx(-st["u"], rel=1e-14)
    assert qg2[0] == pytest.approx(qg[0], rel=1e-14) and qg2[1] == pytest.approx(-qg[1], rel=1e-14)
    # a strong rarefaction: p* is held at the floor, and the linearised star
    # density stays at rho (1 + (p* - p) / (gamma p)) >= (1 - 1/gamma) rho > 0
    qL = np.array([1.0, -3.0, 0.0, 0.0, 1.0])
    qR = np.array([1.0, 3.0, 0.0, 0.0, 1.0])
    _, st, _ = oracle.riemann(qL, qR, LIN)
    assert st["p"] == 1e-20
    assert st["rhoL"] == pytest.approx(1.0 - 1.0 / G, rel=1e-14)
    assert st["rhoR"] == pytest.approx(1.0 - 1.0 / G, rel=1e-14)


def test_linear_solver_step_runs_and_tube_converges():
    def tube(N, t_end=0.2):
        prm = LIN
        shape = (4, 4, N)
        xc = (np.arange(N) + 0.5) / N
        left = np.broadcast_to(xc < 0.5, shape)
        rho = np.where(left, 1.0, 0.125)
        p = np.where(left, 1.0, 0.1)
        U = synth.pad_periodic(synth.conserved(rho, np.zeros((3,) + shape), p, 1.0, 1.4))
        synth.fill_outflow_inplace(U, NG, 0)
        g = np.zeros((3,) + U.shape[1:])
        t, iters = 0.0, 0
        prm = oracle.Params(gamma=1.4, riemann=oracle.RIEMANN_LINEAR)
        while t < t_end - 1e-14:
            dt = min(oracle.estimate_dt(U, NG, 1.0, 1.0 / N, 0.5, prm), t_end - t)
            U, st = oracle.hydro_step(U, g, NG, dt, 1.0 / N, 1.0, 1.0, prm)
            iters += st["riemann_iters"]
            synth.fill_outflow_inplace(U, NG, 0)
            t += dt
        ex = sample(1.0, 0.0, 1.0, 0.125, 0.0, 0.1, 1.4, (xc - 0.5) / t_end)
        line = _valid(U)[0][0, 0]
        return np.abs(line - ex[0]).mean() / np.abs(ex[0]).mean(), iters

    e64, it64 = tube(64)
    e128, _ = tube(128)
    assert it64 == 0
    assert e128 < e64 < 3e-2, (e64, e128)


# ------------------------------------------------ gravity energy form 2 ----

def test_form2_uniform_gas_at_rest_in_uniform_gravity():
    # m^{n+1} = dt rho g; E rises by exactly the kinetic energy gained,
    # |m|^2 / (2 rho); e is unchanged
    rho, p, a0, a1, dt = 1.7, 0.8, 0.5, 0.503, 0.02
    gv = (0.3, -0.2, 0.5)
    shape = (8, 8, 8)
    U = synth.pad_periodic(synth.conserved(np.full(shape, rho), np.zeros((3,) + shape),
                                           np.full(shape, p), a0))
    g = synth.pad_periodic(np.stack([np.full(shape, x) for x in gv]))
    out, _ = oracle.hydro_step(U, g, NG, dt, 1.0 / 8, a0, a1, GF2)
    v = _valid(out)
    m = np.array([dt * rho * x for x in gv])
    for d in range(3):
        assert np.allclose(v[1 + d], m[d], rtol=1e-14, atol=0)
    UE0 = a0 * a0 * p / (G - 1)
    ke = 0.5 * (m * m).sum() / rho
    assert np.allclose(v[4] - UE0, ke, rtol=1e-9)
    assert np.allclose(v[5], UE0, rtol=1e-14)


def test_form2_leaves_mass_and_momentum_and_changes_only_energy():
    w = synth.config1(n=12, seed=31)
    dt = oracle.estimate_dt(w.state, NG, w.a0, w.dx, 0.5)
    f1, _ = oracle.hydro_step(w.state, w.grav, NG, dt, w.dx, w.a0, w.a_at(1))
    f2, _ = oracle.hydro_step(w.state, w.grav, NG, dt, w.dx, w.a0, w.a_at(1), GF2)
    v1, v2 = _valid(f1), _valid(f2)
    for c in range(4):
        assert np.array_equal(v1[c], v2[c]), c
    assert not np.array_equal(v1[4], v2[4])
    # without gravity the two forms coincide exactly
    g0 = np.zeros_like(w.grav)
    h1, _ = oracle.hydro_step(w.state, g0, NG, dt, w.dx, w.a0, w.a_at(1))
    h2, _ = oracle.hydro_step(w.state, g0, NG, dt, w.dx, w.a0, w.a_at(1), GF2)
    assert np.array_equal(_valid(h1), _valid(h2))


def test_form2_energy_change_is_the_gravity_kinetic_energy_change():
    # Both forms share the fluxes (g enters them only through the edge
    # states), the density and the momenta; only the energy's gravity term
    # differs.  From the inputs and outputs alone, with m_h the momentum before
    # the gravity terms and m* after the predictor's:
    #   form 1 adds dt m^n.g + dt/2 (m* - m^n).g,
    #   form 2 adds |m^{n+1}|^2/(2 rho*) - |m_h|^2/(2 rho*),
    # so E_2 - E_1 is the difference of the two terms.
    w = synth.config1(n=10, seed=41)
    dt = oracle.estimate_dt(w.state, NG, w.a0, w.dx, 0.5)
    o1, s1 = oracle.hydro_step(w.state, w.grav, NG, dt, w.dx, w.a0, w.a_at(1))
    o2, s2 = oracle.hydro_step(w.state, w.grav, NG, dt, w.dx, w.a0, w.a_at(1), GF2)
    assert s1["sync_E_from_e"] == 0 and s2["sync_E_from_e"] == 0
    u0, v1, v2, g = _valid(w.state), _valid(o1), _valid(o2), _valid(w.grav)
    rho0, m0, rho1, m1 = u0[0], u0[1:4], v1[0], v1[1:4]
    mh = m1 - ((0.5 * dt) * (rho1 - rho0) + dt * rho0) * g
    ms = mh + (dt * rho0) * g
    form1 = dt * (m0 * g).sum(axis=0) + (0.5 * dt) * ((ms - m0) * g).sum(axis=0)
    form2 = 0.5 * ((m1 * m1).sum(axis=0) - (mh * mh).sum(axis=0)) / rho1
    scale = np.abs(v1[4]).max()
    assert np.abs((v2[4] - v1[4]) - (form2 - form1)).max() <= 1e-12 * scale
    assert np.abs(form2 - form1).max() > 1e-9 * scale  # the forms do differ here


@pytest.mark.parametrize("bad", [dict(recon=2), dict(riemann=3), dict(grav_form=0)])
def test_unknown_variant_is_rejected(bad):
    w = synth.config1(n=8, seed=1)
    with pytest.raises(Exception):
        oracle.hydro_step(w.state, w.grav, NG, 1e-3, w.dx, w.a0, w.a_at(1), oracle.Params(**bad))
