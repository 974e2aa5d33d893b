"""Pins of the oracle's transverse-correction energy path (O7: the internal
energy equation of the corrected edge state, its dual-energy switch and the
revert rule) and of the time-centred scale factor in the tracing Courant
number k_h = dt / (a_h dx).  Each test is built so that one plausible slip in
those places breaks an exact identity, a closed form or a convergence rate:

  * the sign of the p div u term of O7's internal-energy correction, or
    dropping that correction, spoils the second-order agreement of the
    e-driven and E-driven solutions of a diagonal sound wave;
  * taking E - KE where the switch picks e leaves round-off of the kinetic
    energy in the pressure of a Mach 1000 contact;
  * accepting a corrected state with rho <= 0 sends it into the Riemann
    solver, and the step goes non-finite;
  * a_old instead of a_h in k_h moves the one-step density of a quadratic
    profile by about 1e-6 of itself.

Sec. 3.2 (the unsplit method with full corner coupling, the dual-energy
formulation), Sec. 3.6 Steps 2 and 6 (update and dual-energy rule with
threshold 1e-4), Sec. 3.1 (a linear in t within a step).
"""
import math

import numpy as np
import pytest

import oracle
from paper_1301_4498_amd import synth

NG = 4
G = 5.0 / 3.0


def _valid(f):
    return f[:, NG:-NG, NG:-NG, NG:-NG]


# ---------------- O7 e-branch: hypersonic contact ------------------------

def test_hypersonic_contact_keeps_pressure_and_velocity_exactly():
    # A pressure-equilibrium contact (random density, uniform p and U)
    # moving diagonally at Mach 1000.  Its internal energy is about 2e-6 of
    # the total, below the 1e-4 threshold, so every transverse correction
    # (O7) and the final sync (O12) must recover p from the internal-energy
    # equation.  There the density jumps carry no e flux and no p div u
    # term, so p and U stay what they were to round-off.  Recovering p from
    # E - KE instead leaves about 1e-16 of the kinetic energy, i.e. ~1e-10 of
    # p, which the advective e flux carries into the cells.
    n = 8
    rng = np.random.default_rng(5)
    shape = (n, n, n)
    rho = np.exp(rng.normal(0.0, 0.5, shape))
    p0 = 1.0
    c = math.sqrt(G * p0 / rho.min())
    U0 = np.array([0.6, 0.5, 0.62])
    U0 = U0 / np.linalg.norm(U0) * 1000.0 * c
    u = np.stack([np.full(shape, x) for x in U0])
    a = 0.7
    U = synth.pad_periodic(synth.conserved(rho, u, np.full(shape, p0), a))
    g = np.zeros((3,) + U.shape[1:])
    syncs = 0
    for _ in range(2):
        dt = oracle.estimate_dt(U, NG, a, 1.0 / n, 0.5)
        U, st = oracle.hydro_step(U, g, NG, dt, 1.0 / n, a, a)
        synth.fill_periodic_inplace(U)
        syncs += st["sync_E_from_e"]
        assert st["trans_reverts"] == 0 and st["nonfinite"] == 0
    v = _valid(U)
    p = v[5] * (G - 1.0) / (a * a)
    assert np.abs(p / p0 - 1.0).max() <= 1e-13, np.abs(p / p0 - 1.0).max()
    for d in range(3):
        ud = v[1 + d] / (a * v[0])
        assert np.abs(ud / U0[d] - 1.0).max() <= 1e-13
    # the e-branch of the final sync ran in every cell of both steps
    assert syncs == 2 * n ** 3


# ---------------- O7 internal-energy correction: diagonal sound wave ------

def _diagonal_wave_pressure(N, eta, a0=0.5, a1=0.6, t_end=0.1):
    # a sound wave travelling along (1, 1, 0) on an N x N x 2 periodic box,
    # so that x and y are each the other's transverse direction
    shape = (2, N, N)
    h = 1.0 / N
    x = (np.arange(N) + 0.5) * h
    ph = 2.0 * np.pi * (x[None, None, :] + x[None, :, None])
    eps = 0.05
    rho = np.broadcast_to(1.0 + eps * np.sin(ph), shape).copy()
    p0 = 0.6
    c0 = math.sqrt(G * p0)
    p = np.broadcast_to(p0 * (1.0 + G * eps * np.sin(ph)), shape).copy()
    un = np.broadcast_to(c0 * eps * np.sin(ph) / math.sqrt(2.0), shape).copy()
    u = np.stack([un, un.copy(), np.zeros(shape)])
    U = synth.pad_periodic(synth.conserved(rho, u, p, a0))
    g = np.zeros((3,) + U.shape[1:])
    prm = oracle.Params(eta=eta)
    adot = (a1 - a0) / t_end
    t, a = 0.0, a0
    while t < t_end - 1e-14:
        dt = min(oracle.estimate_dt(U, NG, a, h, 0.5), t_end - t)
        an = a0 + adot * (t + dt)
        U, _ = oracle.hydro_step(U, g, NG, dt, h, a, an, prm)
        synth.fill_periodic_inplace(U)
        t += dt
        a = an
    return _valid(U)[5][0] * (G - 1.0) / (a * a)


def test_dual_energy_consistency_on_a_diagonal_wave():
    # eta = 2 makes every switch (O7 and O12) take the internal-energy
    # equation, including its p div u term and, in O7, the transverse e-flux
    # differences; eta = 1e-4 takes E - KE.  Both discretise the same
    # adiabatic flow under expansion, so their pressures must agree at
    # second order.  A wrong sign of O7's p div u term, or an uncorrected
    # internal energy, makes the e-driven edge states first-order wrong.
    diffs = []
    for N in (16, 32, 64):
        pe = _diagonal_wave_pressure(N, 2.0)
        pE = _diagonal_wave_pressure(N, 1e-4)
        diffs.append(np.abs(pe - pE).mean() / np.abs(pE).mean())
    orders = [math.log2(diffs[i] / diffs[i + 1]) for i in range(2)]
    assert min(orders) >= 1.8, (diffs, orders)


# ---------------- O7 revert rule ------------------------------------------

def test_transverse_revert_keeps_the_step_finite():
    # Density rising 16-fold per cell along x (a sawtooth of period 4) makes
    # the low x-edge of each cell about a quarter of the cell's density,
    # while the flow diverges at Mach 20 in y and in z.  The stage-2
    # correction of those x-edges by both transverse flux differences then
    # removes more mass than the edge holds: the corrected density is
    # negative, and O7 must keep the uncorrected edge (counted).  Fed to the
    # Riemann solver, a negative density gives a negative impedance C and
    # the step turns non-finite.
    n = 16
    shape = (n, n, n)
    i = np.arange(n)
    rho = np.broadcast_to((16.0 ** (i % 4))[None, None, :], shape).copy()
    pval = 1e-3
    p = np.full(shape, pval)
    c = math.sqrt(G * pval / rho.min())
    sgn = np.where(i < n // 2, -1.0, 1.0)
    uy = np.broadcast_to(sgn[None, :, None], shape)
    uz = np.broadcast_to(sgn[:, None, None], shape)
    u = np.stack([np.zeros(shape), 20.0 * c * uy, 20.0 * c * uz])
    U = synth.pad_periodic(synth.conserved(rho, u, p, 1.0))
    g = np.zeros((3,) + U.shape[1:])
    dt = oracle.estimate_dt(U, NG, 1.0, 1.0 / n, 0.5)
    out, st = oracle.hydro_step(U, g, NG, dt, 1.0 / n, 1.0, 1.0)
    v = _valid(out)
    assert st["trans_reverts"] > 0
    assert st["nonfinite"] == 0 and np.isfinite(v).all()
    assert st["neg_dens"] == 0 and v[0].min() > 0.0
    assert st["neg_eint"] == 0 and v[5].min() > 0.0


# ---------------- k_h centring: quadratic density, one step --------------

@pytest.mark.parametrize("a_pair", [(1.0, 1.0), (0.5, 0.51), (0.25, 0.2575)])
def test_quadratic_density_one_step_closed_form(a_pair):
    # rho(x) = 1 + b x + c x^2 (cell averages, ghosts included, so no
    # boundary is seen), uniform U and p, no gravity, uniform in y and z.
    # PPM reproduces a quadratic exactly, so the traced edge density of the
    # face at x_f is the exact average of rho over the upwind distance
    # sigma h, sigma = U k_h, k_h = dt / (a_h dx), and the half-step
    # expansion term slows the edge velocity to u_e = U (1 - da / (2 a_h)).
    # The face is a contact, so the Godunov state is that edge state, and
    #   rho' = rho - (dt/dx) (u_e / a_h) (avg_{j+1/2} - avg_{j-1/2}),
    #   m'   = m   - (dt/dx) u_e^2 (avg_{j+1/2} - avg_{j-1/2}).
    # The averages come from the antiderivative, not from the scheme's own
    # parabola formula.
    a0, a1 = a_pair
    n = 16
    h = 1.0 / n
    bq, cq = 0.5, 0.3

    def prim(x):  # antiderivative of rho
        return x + bq * x * x / 2.0 + cq * x ** 3 / 3.0

    def avg(xl, xr):
        return (prim(xr) - prim(xl)) / (xr - xl)

    xs = np.arange(-NG, n + NG) * h
    rho1 = avg(xs, xs + h)
    sh = (2 + 2 * NG, 2 + 2 * NG, n + 2 * NG)
    rho = np.broadcast_to(rho1[None, None, :], sh).copy()
    Uv, p0 = 0.4, 0.8
    u = np.stack([np.full(sh, Uv), np.zeros(sh), np.zeros(sh)])
    U = np.ascontiguousarray(synth.conserved(rho, u, np.full(sh, p0), a0))
    g = np.zeros((3,) + sh)
    dt = 0.4 * h * a0 / (Uv + math.sqrt(G * p0 / rho.min()))
    out, st = oracle.hydro_step(U, g, NG, dt, h, a0, a1)
    ah = 0.5 * (a0 + a1)
    sig = Uv * (dt / (ah * h))
    ue = Uv * (1.0 - (a1 - a0) / (2.0 * ah))
    xf = np.arange(n + 1) * h  # faces 0..n
    face = avg(xf - sig * h, xf)
    k = dt / h
    want_rho = rho1[NG:-NG] - k * (ue / ah) * (face[1:] - face[:-1])
    want_m = a0 * rho1[NG:-NG] * Uv - k * ue * ue * (face[1:] - face[:-1])
    got = _valid(out)
    assert np.abs(got[0] / want_rho - 1.0).max() <= 1e-13, np.abs(got[0] / want_rho - 1.0).max()
    assert np.abs(got[1] / want_m - 1.0).max() <= 1e-13, np.abs(got[1] / want_m - 1.0).max()
    assert st["trans_reverts"] == 0
