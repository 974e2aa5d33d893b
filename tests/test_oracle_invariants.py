"""Whole-step pins of the oracle: closed forms of Sec. 3.2 / 3.6, conservation,
axis-permutation symmetry, Galilean special cases, expansion rescaling, the
dual-energy branch and the CFL formula of Sec. 3.5 (no GPU)."""
import math

import numpy as np
import pytest

import oracle
from paper_1301_4498_amd import synth

NG = 4
P = oracle.Params()
G = P.gamma


def _uniform(n, rho, u, p, a, g=(0.0, 0.0, 0.0)):
    nx, ny, nz = n
    shape = (nz, ny, nx)
    U = synth.conserved(np.full(shape, rho), np.stack([np.full(shape, x) for x in u]),
                        np.full(shape, p), a)
    gg = np.stack([np.full(shape, x) for x in g])
    return synth.pad_periodic(U), synth.pad_periodic(gg)


def _valid(f):
    return f[:, NG:-NG, NG:-NG, NG:-NG]


def test_uniform_state_is_preserved():
    U, g = _uniform((8, 6, 10), 1.3, (0.4, -0.7, 0.2), 0.9, 0.7)
    out, st = oracle.hydro_step(U, g, NG, 0.01, 0.1, 0.7, 0.7)
    assert np.allclose(_valid(out), _valid(U), rtol=1e-13, atol=0)
    assert st["riemann_calls"] > 0 and st["trans_reverts"] == 0


def test_uniform_gas_at_rest_in_uniform_gravity():
    # predictor + corrector with zero flux divergence (Sec. 3.6 Steps 2, 6):
    # m^{n+1} = dt rho g,  dU_E = dt^2 rho |g|^2 / 2,  U_e unchanged
    rho, p, a0, a1, dt = 1.7, 0.8, 0.5, 0.503, 0.02
    gv = (0.3, -0.2, 0.5)
    U, g = _uniform((8, 8, 8), rho, (0, 0, 0), p, a0, gv)
    out, st = oracle.hydro_step(U, g, NG, dt, 1.0 / 8, a0, a1)
    v = _valid(out)
    for d in range(3):
        assert np.allclose(v[1 + d], dt * rho * gv[d], rtol=1e-14, atol=0)
    g2 = sum(x * x for x in gv)
    UE0 = a0 * a0 * p / (G - 1)
    assert np.allclose(v[4] - UE0, 0.5 * dt * dt * rho * g2, rtol=1e-9)
    assert np.allclose(v[4], UE0 + 0.5 * dt * dt * rho * g2, rtol=1e-14)
    assert np.allclose(v[5], UE0, rtol=1e-14)
    assert np.all(v[0] == rho)


def test_uniform_moving_gas_under_expansion():
    # gamma = 5/3: with no gradients the stored U is constant, i.e. peculiar
    # velocity ~ 1/a and energies ~ 1/a^2 (Sec. 2.2 simplified equations)
    U, g = _uniform((6, 6, 6), 0.9, (0.5, 0.25, -0.4), 0.3, 0.25)
    out, _ = oracle.hydro_step(U, g, NG, 0.01, 1.0 / 6, 0.25, 0.26)
    assert np.allclose(_valid(out), _valid(U), rtol=1e-14, atol=0)


def test_conservation_periodic_no_gravity():
    w = synth.config1(n=16, seed=21)
    g = np.zeros_like(w.grav)
    dt = oracle.estimate_dt(w.state, NG, w.a0, w.dx, 0.5)
    out, st = oracle.hydro_step(w.state, g, NG, dt, w.dx, w.a0, w.a0 * 1.01)
    assert st["sync_E_from_e"] == 0  # that branch breaks energy conservation by design
    v0, v1 = _valid(w.state), _valid(out)
    for c in range(5):
        s0 = math.fsum(v0[c].ravel())
        s1 = math.fsum(v1[c].ravel())
        scale = math.fsum(np.abs(v0[c]).ravel())
        assert abs(s1 - s0) <= 1e-13 * scale, (c, s0, s1)


def _perm(f, is_vec_state):
    """Cyclic relabelling new x = old y, new y = old z, new z = old x."""
    t = f.transpose(0, 3, 1, 2)
    if is_vec_state:
        return np.ascontiguousarray(t[[0, 2, 3, 1, 4, 5]])
    return np.ascontiguousarray(t[[1, 2, 0]])


def test_axis_permutation_commutes_with_step():
    U, g = synth.random_box((8, 10, 12), seed=4, a=0.5)
    dt = oracle.estimate_dt(U, NG, 0.5, 1 / 16, 0.5)
    out, _ = oracle.hydro_step(U, g, NG, dt, 1 / 16, 0.5, 0.505)
    out2, _ = oracle.hydro_step(_perm(U, True), _perm(g, False), NG, dt, 1 / 16, 0.5, 0.505)
    a, b = _valid(_perm(out, True)), _valid(out2)
    for c in range(6):
        rel = np.abs(a[c] - b[c]).sum() / np.abs(a[c]).sum()
        assert rel <= 1e-13, (c, rel)


def test_galilean_uniform_boost():
    # G1: any uniform velocity keeps a uniform state uniform
    for u in [(3.0, 0, 0), (0, -5.0, 0), (1.0, 2.0, -3.0)]:
        U, g = _uniform((8, 8, 8), 0.6, u, 1.1, 1.0)
        out, _ = oracle.hydro_step(U, g, NG, 0.005, 1 / 8, 1.0, 1.0)
        assert np.allclose(_valid(out), _valid(U), rtol=1e-13, atol=1e-14)


def test_galilean_contact_keeps_pressure_and_velocity():
    # G2: a pressure-equilibrium contact: density varies, p and U constant
    n = (16, 8, 8)
    rng = np.random.default_rng(8)
    shape = (n[2], n[1], n[0])
    rho = np.exp(rng.normal(0, 0.5, shape))
    u = np.stack([np.full(shape, 0.7), np.full(shape, -0.3), np.full(shape, 0.2)])
    p = np.full(shape, 1.3)
    U = synth.pad_periodic(synth.conserved(rho, u, p, 1.0))
    g = np.zeros((3,) + U.shape[1:])
    for _ in range(3):
        dt = oracle.estimate_dt(U, NG, 1.0, 1 / 16, 0.5)
        U, st = oracle.hydro_step(U, g, NG, dt, 1 / 16, 1.0, 1.0)
        synth.fill_periodic_inplace(U)
    v = _valid(U)
    for d, ud in enumerate((0.7, -0.3, 0.2)):
        assert np.allclose(v[1 + d] / v[0], ud, rtol=1e-13, atol=1e-14)
    pe = (G - 1) * v[5]
    pE = (G - 1) * (v[4] - 0.5 * (v[1] ** 2 + v[2] ** 2 + v[3] ** 2) / v[0])
    assert np.allclose(pe, 1.3, rtol=1e-13) and np.allclose(pE, 1.3, rtol=1e-12)


def _entropy_wave_error(N, U0=1.0, t_end=0.25):
    n = (N, 2, 2)
    x = (np.arange(N) + 0.5) / N
    shape = (2, 2, N)

    def rho_avg(xc, t):
        # exact cell average of 1 + 0.2 sin(2 pi (x - U0 t))
        h = 1.0 / N
        return 1.0 + 0.2 * (np.cos(2 * np.pi * (xc - h / 2 - U0 * t)) -
                            np.cos(2 * np.pi * (xc + h / 2 - U0 * t))) / (2 * np.pi * h)

    rho = np.broadcast_to(rho_avg(x, 0.0), shape).copy()
    u = np.stack([np.full(shape, U0), np.zeros(shape), np.zeros(shape)])
    p = np.ones(shape)
    U = synth.pad_periodic(synth.conserved(rho, u, p, 1.0))
    g = np.zeros((3,) + U.shape[1:])
    t = 0.0
    while t < t_end - 1e-14:
        dt = min(oracle.estimate_dt(U, NG, 1.0, 1.0 / N, 0.5), t_end - t)
        U, _ = oracle.hydro_step(U, g, NG, dt, 1.0 / N, 1.0, 1.0)
        synth.fill_periodic_inplace(U)
        t += dt
    r = _valid(U)[0][0, 0]
    return np.abs(r - rho_avg(x, t_end)).mean()


def test_galilean_boosted_entropy_wave_converges():
    # G3: second-order convergence of a boosted entropy wave (exact translation)
    errs = [_entropy_wave_error(N) for N in (32, 64, 128)]
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert errs[0] < 2e-3
    assert min(orders) >= 1.8, (errs, orders)


def test_constant_a_equals_unit_a_with_rescaled_dt():
    # with a fixed, the comoving equations are Euler in tau = t/a (Sec. 2.2)
    a = 0.7
    nx = ny = nz = 8
    rng = np.random.default_rng(12)
    shape = (nz, ny, nx)
    rho = synth.lognormal(rng, shape, 1.0, 0.4)
    u = rng.normal(0, 0.3, (3,) + shape)
    p = synth.lognormal(rng, shape, 0.6, 0.3)
    gg = synth.pad_periodic(rng.normal(0, 0.05, (3,) + shape))
    Ua = synth.pad_periodic(synth.conserved(rho, u, p, a))
    U1 = synth.pad_periodic(synth.conserved(rho, u, p, 1.0))
    dt = 0.004
    outa, _ = oracle.hydro_step(Ua, gg, NG, dt, 1 / 8, a, a)
    out1, _ = oracle.hydro_step(U1, gg, NG, dt / a, 1 / 8, 1.0, 1.0)
    va, v1 = _valid(outa), _valid(out1)
    assert np.allclose(va[0], v1[0], rtol=1e-13)
    for d in range(3):
        assert np.allclose(va[1 + d] / (a * va[0]), v1[1 + d] / v1[0], rtol=1e-12, atol=1e-14)
    assert np.allclose(va[5] / (a * a), v1[5], rtol=1e-12)


def test_dual_energy_branch_selection():
    # Sec. 3.6 Step 6: e/E below 1e-4 -> E rebuilt from e; above -> e from E
    for ratio, expect_sync in ((0.5e-4, True), (2e-4, False)):
        rho, u = 1.0, 10.0
        ke = 0.5 * rho * u * u
        # (E - KE)/E = ratio with E = KE + rho e
        rhoe = ratio * ke / (1 - ratio)
        p = (G - 1) * rhoe
        U, g = _uniform((4, 4, 4), rho, (u, 0, 0), p, 1.0)
        out, st = oracle.hydro_step(U, g, NG, 1e-4, 0.25, 1.0, 1.0)
        assert (st["sync_E_from_e"] == 64) == expect_sync
        assert (st["sync_E_from_e"] == 0) == (not expect_sync)


def test_cfl_closed_form_uniform_state():
    rho, u, p, a, dx = 1.4, (0.3, -1.2, 0.8), 0.7, 0.6, 1 / 32
    U, _ = _uniform((8, 8, 8), rho, u, p, a)
    dt = oracle.estimate_dt(U, NG, a, dx, 0.5)
    c = math.sqrt(G * p / rho)
    assert dt == pytest.approx(0.5 * a * dx / (max(abs(x) for x in u) + c), rel=1e-15)


def test_cfl_ignores_ghost_cells():
    U, _ = synth.random_box((8, 8, 8), seed=2, a=0.5)
    dt0 = oracle.estimate_dt(U, NG, 0.5, 1 / 8, 0.5)
    U2 = U.copy()
    U2[1, :NG] = 1e6  # huge momentum in ghosts only
    assert oracle.estimate_dt(U2, NG, 0.5, 1 / 8, 0.5) == dt0
