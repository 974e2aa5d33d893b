"""The operation-count build of the oracle (oracle/opcount.cpp) against
counts derived by hand from the formulas it evaluates, and against the plain
oracle's results (it must compute the same bits)."""
import numpy as np
import pytest

import oracle
from oracle import opcount
from paper_1301_4498_amd import synth

NG = 4


@pytest.fixture(scope="module", autouse=True)
def _built():
    opcount.build(force=False)


def test_counting_build_computes_the_oracle_bits():
    U, g = synth.random_box((12, 10, 8), seed=41, a=0.5)
    dx = 1.0 / 12
    dt = oracle.estimate_dt(U, NG, 0.5, dx, 0.5)
    ref, st = oracle.hydro_step(U, g, NG, dt, dx, 0.5, 0.505)
    out, st2, _ = opcount.count_step(U, g, NG, dt, dx, 0.5, 0.505)
    assert np.array_equal(out, ref)
    assert st == st2
    dt2, _ = opcount.count_dt(U, NG, 0.5, dx, 0.5)
    assert dt2 == dt


def test_cfl_counts_closed_form():
    # per valid cell (Sec. 3.5 formula as the oracle writes it):
    #   re = U_e / (a a)             1 mul, 1 div
    #   p = max(gm1 re, small)       1 mul, 1 cmp
    #   c = sqrt((gamma p) / rho)    1 mul, 1 div, 1 sqrt;   rho floor: 1 cmp
    #   per d: |m_d / (a rho)| + c   1 mul, 1 div, 1 add;    max: 1 cmp
    # once: gm1 = gamma - 1 (1 add); dt = ((cfl a) dx) / smax (2 mul, 1 div)
    n = (9, 7, 5)
    U, _ = synth.random_box(n, seed=3, a=0.7)
    V = 9 * 7 * 5
    _, c = opcount.count_dt(U, NG, 0.7, 0.1, 0.5)
    add, mul, div, sq, cmp_ = c[8].sum(axis=0)
    assert (add, mul, div, sq, cmp_) == (3 * V + 1, 6 * V + 2, 5 * V + 1, V, 5 * V)


def test_primitive_counts_closed_form():
    # O1 per padded cell: u_d = U_d / (a_old rho): 2 x 3; rho e = U_e /
    # (a_old a_old): 2; p = gm1 rho e: 1; c = sqrt((gamma p) / rho): 3 -> 12
    n = (6, 6, 6)
    U, g = synth.random_box(n, seed=8, a=0.5)
    dt = oracle.estimate_dt(U, NG, 0.5, 1 / 6, 0.5)
    _, _, c = opcount.count_step(U, g, NG, dt, 1 / 6, 0.5, 0.5)
    P = 14 ** 3
    assert opcount.flops(c[1]) == 12 * P
    assert c[1][1].sum() == 0  # no Riemann solve in O1


def test_newton_iteration_counts():
    # one pass of the two-shock Newton loop (O5):
    #   W_K = sqrt(C_K + (g2 rho_K)(p - p_K))  5 x 2
    #   u*_K = u_K -/+ (p - p_K) / W_K         3 x 2
    #   Z_K = ((2 W) W) W / (W W + C)           6 x 2
    #   p' = p - ((Z_L Z_R)(u*_R - u*_L)) / (Z_L + Z_R)   6
    #   stop test |p' - p| <= tol p'            2
    # = 36 flops, 2 square roots; the stages' iteration totals equal the
    # oracle's own iteration counter
    U, g = synth.random_box((8, 8, 8), seed=5, a=0.5)
    dt = oracle.estimate_dt(U, NG, 0.5, 1 / 8, 0.5)
    _, st, c = opcount.count_step(U, g, NG, dt, 1 / 8, 0.5, 0.505)
    it = c[4:7, 1]  # stages 0, 1, 2 inside iterations
    iters = int(it[:, 3].sum()) // 2
    assert iters == st["riemann_iters"]
    assert int(it[:, :4].sum()) == 36 * iters
    # the Riemann solves happen only in the three Riemann stages
    assert c[:4, 1].sum() == 0 and c[7:, 1].sum() == 0
