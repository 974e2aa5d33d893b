"""Pins of the oracle's building blocks against closed forms, special cases
and an independent exact Riemann solver (no GPU)."""
import math

import numpy as np
import pytest

import oracle
from exact_riemann import sample, star_state

P = oracle.Params()


# ---------------- PPM (O3) ----------------

def _cell_avgs_cubic(coef, xs, h):
    """Exact cell averages of a cubic over [x - h/2, x + h/2]."""
    c0, c1, c2, c3 = coef
    F = lambda x: c0 * x + c1 * x**2 / 2 + c2 * x**3 / 3 + c3 * x**4 / 4
    return (F(xs + h / 2) - F(xs - h / 2)) / h


def test_ppm_interface_exact_on_cubic_averages():
    # monotone cubic with the slope limiter inactive: the interface value is the
    # fourth-order formula 7/12 (q_j + q_j+1) - 1/12 (q_j-1 + q_j+2), exact for cubics
    coef = (1.0, 0.8, 0.1, 0.05)
    h = 0.1
    xs = np.arange(-5, 5) * h
    q = _cell_avgs_cubic(coef, xs, h)
    for j in range(1, len(xs) - 2):
        v = oracle.ppm_interface(q[j - 1:j + 3])
        xe = xs[j] + h / 2
        exact = coef[0] + coef[1] * xe + coef[2] * xe**2 + coef[3] * xe**3
        assert abs(v - exact) <= 1e-13 * abs(exact)
        # and the closed-form combination of averages
        four = 7.0 / 12.0 * (q[j] + q[j + 1]) - 1.0 / 12.0 * (q[j - 1] + q[j + 2])
        assert abs(v - four) <= 1e-14 * abs(four)


def test_ppm_constant_data_bitwise():
    q = np.full(12, 0.7312)
    qm, qp = oracle.ppm_line(q)
    assert np.all(qm[2:-2] == 0.7312) and np.all(qp[2:-2] == 0.7312)


def test_ppm_extremum_is_flattened_to_constant():
    # a local maximum at cell j: (q+ - q_j)(q_j - q-) <= 0 -> both edges = q_j
    q = np.array([0.0, 1.0, 2.0, 3.0, 5.0, 3.0, 2.0, 1.0, 0.0])
    qm, qp = oracle.ppm_line(q)
    assert qm[4] == 5.0 and qp[4] == 5.0


def test_ppm_monotone_profile_stays_within_neighbours():
    rng = np.random.default_rng(11)
    q = np.cumsum(rng.uniform(0.0, 1.0, 40))
    q[20:] += 10.0  # a jump
    qm, qp = oracle.ppm_line(q)
    for j in range(2, 38):
        lo, hi = min(q[j - 1], q[j + 1]), max(q[j - 1], q[j + 1])
        assert lo - 1e-12 <= qm[j] <= hi + 1e-12
        assert lo - 1e-12 <= qp[j] <= hi + 1e-12


def test_ppm_chi_zero_gives_piecewise_constant():
    rng = np.random.default_rng(3)
    q = rng.uniform(1, 2, 16)
    qm, qp = oracle.ppm_line(q, np.zeros(16))
    assert np.all(qm[2:-2] == q[2:-2]) and np.all(qp[2:-2] == q[2:-2])


# ---------------- flattening (O2) ----------------

def test_flatten_smooth_data_is_one():
    x = np.linspace(0, 1, 20)
    p = 1.0 + 0.01 * np.sin(2 * np.pi * x)
    u = -0.1 * x  # compressive, but the pressure jump is tiny
    chi = oracle.flatten_line(p, u)
    assert np.all(chi[3:-3] == 1.0)


def test_flatten_strong_compressive_jump_is_zero():
    p = np.array([1.0] * 6 + [10.0] * 6)
    u = np.array([1.0] * 6 + [0.0] * 6)
    chi = oracle.flatten_line(p, u)
    # cells 5 and 6 straddle the jump; z = 1 -> omega2 (1 - omega1) > 1 -> f~ = 1
    assert chi[5] == 0.0 and chi[6] == 0.0
    # an expanding flow with the same jump is not flattened
    chi2 = oracle.flatten_line(p, -u)
    assert np.all(chi2[3:-3] == 1.0)


def test_flatten_takes_low_pressure_neighbour():
    # f~ nonzero at cell 5 only (jump between 5 and 6 seen by 4..6); cell 4 has
    # dp1 = p5 - p3 > 0 so it takes max(f~4, f~3): unaffected by cell 5
    p = np.array([1, 1, 1, 1, 1, 1, 4, 4, 4, 4, 4, 4], dtype=float)
    u = np.array([1, 1, 1, 1, 1, 1, 0, 0, 0, 0, 0, 0], dtype=float)
    chi = oracle.flatten_line(p, u)
    # cell 7: dp1 = p8 - p6 = 0 -> own f~ only; cell 6: dp1 = p7 - p5 > 0 ->
    # max(f~6, f~5)
    assert chi[7] == 1.0
    assert chi[6] == chi[5] < 1.0


# ---------------- tracing (O4) ----------------

def test_trace_constant_profile_returns_constant():
    qc = np.array([1.3, 0.2, -0.1, 0.05, 0.9])
    c = math.sqrt(P.gamma * qc[4] / qc[0])
    for d in range(3):
        lo, hi = oracle.trace_cell(d, qc, c, qc, qc, np.zeros(3), kh=0.4)
        assert np.all(lo == qc) and np.all(hi == qc)


def test_trace_unit_courant_number_reaches_cell_average():
    # at rest, sigma = c kh = 1: the fastest wave toward each face averages the
    # whole parabola, which is the cell average, so both edge states equal the
    # cell values of rho, u, p whatever the parabola is
    rng = np.random.default_rng(5)
    qc = np.array([1.1, 0.0, 0.0, 0.0, 0.8])
    c = math.sqrt(P.gamma * qc[4] / qc[0])
    dq = rng.uniform(-0.05, 0.05, 5)
    qm = qc - dq
    qp = qc + dq
    qm[1:4] = 0.0
    qp[1:4] = 0.0
    lo, hi = oracle.trace_cell(0, qc, c, qm, qp, np.zeros(3), kh=1.0 / c)
    for v in (0, 1, 4):
        assert abs(lo[v] - qc[v]) <= 1e-15 * max(1, abs(qc[v]))
        assert abs(hi[v] - qc[v]) <= 1e-15 * max(1, abs(qc[v]))


def test_trace_half_step_sources():
    qc = np.array([1.0, 0.3, -0.2, 0.1, 0.6])
    c = math.sqrt(P.gamma * qc[4] / qc[0])
    g = np.array([0.5, -0.25, 0.125])
    lo, hi = oracle.trace_cell(1, qc, c, qc, qc, g, kh=0.3, hdt_a=0.01, hda_a=0.002, pexp=0.004)
    for e in (lo, hi):
        for d in range(3):
            assert e[1 + d] == pytest.approx(qc[1 + d] + 0.01 * g[d] - 0.002 * qc[1 + d], rel=1e-15)
        assert e[4] == pytest.approx(qc[4] - 0.004 * qc[4], rel=1e-15)


# ---------------- two-shock Riemann solver (O5) ----------------

def _colliding_states(rng, n):
    out = []
    for _ in range(n):
        rl, rr = rng.uniform(0.2, 5.0, 2)
        pl, pr = rng.uniform(0.1, 5.0, 2)
        cl, cr = math.sqrt(P.gamma * pl / rl), math.sqrt(P.gamma * pr / rr)
        ul = rng.uniform(1.0, 4.0) * max(cl, cr)
        ur = -rng.uniform(1.0, 4.0) * max(cl, cr)
        out.append(((rl, ul, pl), (rr, ur, pr)))
    return out


def test_two_shock_equals_exact_for_double_shocks():
    rng = np.random.default_rng(42)
    n_checked = 0
    for (rl, ul, pl), (rr, ur, pr) in _colliding_states(rng, 200):
        ps, us = star_state(rl, ul, pl, rr, ur, pr, P.gamma)
        if not (ps > pl and ps > pr):
            continue
        qg, star, it = oracle.riemann([rl, ul, 0.3, -0.2, pl], [rr, ur, 0.1, 0.4, pr])
        assert abs(star["p"] - ps) <= 1e-12 * ps
        assert abs(star["u"] - us) <= 1e-12 * max(abs(us), math.sqrt(ps))
        # Godunov state = exact solution at x/t = 0
        ex = sample(rl, ul, pl, rr, ur, pr, P.gamma, np.array([0.0]))[:, 0]
        assert abs(qg[0] - ex[0]) <= 1e-12 * ex[0]
        assert abs(qg[1] - ex[1]) <= 1e-12 * max(abs(ex[1]), 1.0)
        assert abs(qg[4] - ex[2]) <= 1e-12 * ex[2]
        assert 1 <= it <= 20
        n_checked += 1
    assert n_checked > 150


def test_riemann_mirror_symmetry():
    rng = np.random.default_rng(7)
    for _ in range(200):
        qL = np.array([rng.uniform(0.1, 3), rng.normal(0, 2), rng.normal(), rng.normal(), rng.uniform(0.05, 3)])
        qR = np.array([rng.uniform(0.1, 3), rng.normal(0, 2), rng.normal(), rng.normal(), rng.uniform(0.05, 3)])
        qg, st, _ = oracle.riemann(qL, qR)
        mL = qR * np.array([1, -1, 1, 1, 1])
        mR = qL * np.array([1, -1, 1, 1, 1])
        qg2, st2, _ = oracle.riemann(mL, mR)
        assert st2["p"] == pytest.approx(st["p"], rel=1e-13)
        assert st2["u"] == pytest.approx(-st["u"], rel=1e-12, abs=1e-13)
        if abs(st["u"]) > 1e-10:
            assert qg2[0] == pytest.approx(qg[0], rel=1e-12)
            assert qg2[1] == pytest.approx(-qg[1], rel=1e-12, abs=1e-13)
            assert qg2[4] == pytest.approx(qg[4], rel=1e-12)
            assert qg2[2] == qg[2] and qg2[3] == qg[3]


def test_riemann_equal_states():
    q = np.array([0.7, 0.4, -0.3, 0.2, 1.9])
    qg, st, _ = oracle.riemann(q, q)
    assert st["p"] == pytest.approx(q[4], rel=1e-15)
    assert st["u"] == pytest.approx(q[1], rel=1e-15)
    assert qg == pytest.approx(q, rel=1e-15)


def test_riemann_star_state_satisfies_two_shock_jump_conditions():
    # independent check of the iteration's fixed point: at p*, the shock
    # velocity jumps computed from the Rankine-Hugoniot mass flux agree
    rng = np.random.default_rng(9)
    g = P.gamma
    for _ in range(100):
        rl, rr, pl, pr = rng.uniform(0.1, 4, 4)
        ul, ur = rng.normal(0, 1.5, 2)
        _, st, _ = oracle.riemann([rl, ul, 0, 0, pl], [rr, ur, 0, 0, pr])
        p = st["p"]
        if p <= 1e-12:
            continue
        # Rankine-Hugoniot mass flux for a shock from state K to pressure p
        mK = lambda r, pk: math.sqrt(r * ((g + 1) / 2 * p + (g - 1) / 2 * pk))
        uL = ul - (p - pl) / mK(rl, pl)
        uR = ur + (p - pr) / mK(rr, pr)
        assert abs(uL - uR) <= 1e-12 * (abs(ul) + abs(ur) + math.sqrt(g * max(pl / rl, pr / rr)))
        # Hugoniot density: mass conservation across the left shock
        rsL = st["rhoL"]
        m = mK(rl, pl)
        # 1/rho* = 1/rho - (p - pL)/m^2
        assert 1.0 / rsL == pytest.approx(1.0 / rl - (p - pl) / m**2, rel=1e-12)


def test_exact_solver_self_consistency():
    # the exact solver itself: star state satisfies f_L + f_R + du = 0 and the
    # sampled shock obeys the Rankine-Hugoniot conditions
    g = 1.4
    rl, ul, pl, rr, ur, pr = 1.0, 0.0, 1.0, 0.125, 0.0, 0.1
    ps, us = star_state(rl, ul, pl, rr, ur, pr, g)
    xi = np.linspace(-2, 2, 4001)
    s = sample(rl, ul, pl, rr, ur, pr, g, xi)
    # right shock: find the density jump
    k = np.argmax(np.abs(np.diff(s[0])) * (xi[1:] > us))
    r1, u1, p1 = s[:, k]
    r2, u2, p2 = s[:, k + 1]
    # shock speed from mass conservation, then momentum and energy must balance
    S = (r2 * u2 - r1 * u1) / (r2 - r1)
    assert xi[k] - 2e-3 <= S <= xi[k + 1] + 2e-3
    E1 = p1 / (g - 1) + 0.5 * r1 * u1 * u1
    E2 = p2 / (g - 1) + 0.5 * r2 * u2 * u2
    assert (r1 * u1 * u1 + p1) - S * r1 * u1 == pytest.approx((r2 * u2 * u2 + p2) - S * r2 * u2, rel=1e-12)
    assert u1 * (E1 + p1) - S * E1 == pytest.approx(u2 * (E2 + p2) - S * E2, rel=1e-12, abs=1e-14)
    assert p1 == pytest.approx(ps, rel=1e-12) and u1 == pytest.approx(us, rel=1e-12)
