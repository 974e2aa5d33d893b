"""Pins of the oracle's gravity input path (Sec. 2.4, Sec. 3.4 Self-gravity),
no GPU: the cloud-in-cell deposit equals a brute-force cube/cell overlap
computation and conserves mass; the Poisson solution satisfies the 7-point
equation and single-mode closed forms; the centred gradient is exact on a
single mode; and, as the paper states for this combination of deposit,
centred difference and interpolation, a particle exerts no force on itself
while two particles attract with equal and opposite forces."""
import numpy as np
import pytest

import oracle


def _brute_cic(pos, mass, shape, dx):
    """Overlap volume of each particle's cube with each cell, by interval
    intersection over the 3 x 3 x 3 cells around it (periodic images)."""
    nz, ny, nx = shape
    n = (nx, ny, nz)
    rho = np.zeros(shape)
    for p in range(mass.size):
        x = pos[:, p]
        c = [int(np.floor(x[d] / dx)) for d in range(3)]
        for dk in (-1, 0, 1):
            for dj in (-1, 0, 1):
                for di in (-1, 0, 1):
                    cell = (c[0] + di, c[1] + dj, c[2] + dk)
                    vol = 1.0
                    for d in range(3):
                        lo = max(x[d] - 0.5 * dx, cell[d] * dx)
                        hi = min(x[d] + 0.5 * dx, (cell[d] + 1) * dx)
                        vol *= max(0.0, hi - lo)
                    if vol > 0.0:
                        rho[cell[2] % n[2], cell[1] % n[1], cell[0] % n[0]] += \
                            mass[p] * vol / dx ** 3 / dx ** 3
    return rho


def test_cic_deposit_is_the_cube_cell_overlap():
    rng = np.random.default_rng(3)
    shape, dx = (6, 5, 8), 0.125
    L = np.array([8, 5, 6]) * dx
    pos = rng.uniform(0, 1, (3, 40)) * L[:, None]
    pos[:, :3] = [[0.001, L[0] - 1e-3, 0.5 * dx], [0.0, 0.3, L[1] - 1e-9], [0.2, 0.0, 0.4]]
    mass = rng.uniform(0.5, 2.0, 40)
    rho = oracle.cic_deposit(pos, mass, shape, dx)
    ref = _brute_cic(pos, mass, shape, dx)
    assert np.allclose(rho, ref, rtol=1e-12, atol=1e-12 * ref.max())
    assert abs(rho.sum() * dx ** 3 - mass.sum()) <= 1e-13 * mass.sum()


def test_cic_special_positions():
    shape, dx = (4, 4, 4), 0.25
    # at a cell centre: all the mass in that cell
    rho = oracle.cic_deposit(np.array([[0.375], [0.625], [0.125]]), np.array([2.0]), shape, dx)
    assert rho[0, 2, 1] == 2.0 / dx ** 3 and np.count_nonzero(rho) == 1
    # at a cell corner: one eighth in each of eight cells, across the periodic boundary
    rho = oracle.cic_deposit(np.array([[0.0], [0.5], [0.75]]), np.array([1.0]), shape, dx)
    assert np.count_nonzero(rho) == 8
    assert np.allclose(rho[rho > 0], 0.125 / dx ** 3, rtol=1e-15)
    assert rho[2, 1, 3] > 0 and rho[3, 2, 0] > 0


def test_poisson_solution_satisfies_the_7_point_equation():
    rng = np.random.default_rng(4)
    shape, dx, coef = (8, 12, 16), 1.0 / 16, 3.7
    rho = rng.lognormal(0.0, 0.5, shape)
    phi = oracle.poisson_solve(rho, dx, coef)
    f = coef * (rho - rho.mean())
    r = oracle.laplacian7(phi, dx) - f
    assert np.abs(r).max() <= 1e-11 * np.abs(f).max()
    assert abs(phi.mean()) <= 1e-14 * np.abs(phi).max()
    # the solve is linear and the mean of rho does not matter
    phi2 = oracle.poisson_solve(2.0 * rho + 5.0, dx, coef)
    assert np.allclose(phi2, 2.0 * phi, rtol=0, atol=1e-12 * np.abs(phi).max())


def test_poisson_and_gradient_single_mode_closed_forms():
    nx, dx, m = 32, 1.0 / 32, 3
    x = (np.arange(nx) + 0.5) * dx
    shape = (4, 4, nx)
    rho = np.broadcast_to(np.sin(2 * np.pi * m * x), shape).copy()
    phi = oracle.poisson_solve(rho, dx, 1.0)
    theta = 2 * np.pi * m * dx
    # the 7-point operator's eigenvalue of this mode is (2 cos(theta) - 2) / dx^2
    expect = rho * dx * dx / (2 * np.cos(theta) - 2)
    assert np.allclose(phi, expect, rtol=0, atol=1e-13 * np.abs(expect).max())
    g = oracle.gradient(expect, dx)
    gx = -np.cos(2 * np.pi * m * x) * np.sin(theta) / dx * (dx * dx / (2 * np.cos(theta) - 2))
    assert np.allclose(g[0], np.broadcast_to(gx, shape), rtol=0, atol=1e-12 * np.abs(gx).max())
    assert np.abs(g[1]).max() == 0.0 and np.abs(g[2]).max() == 0.0


def _force(pos_src, m_src, pos_at, shape, dx, coef=1.0):
    rho = oracle.cic_deposit(pos_src, m_src, shape, dx)
    g = oracle.gradient(oracle.poisson_solve(rho, dx, coef), dx)
    return np.stack([oracle.cic_interp(pos_at, g[d], dx) for d in range(3)])


def test_no_self_force_and_equal_and_opposite_pair_forces():
    rng = np.random.default_rng(5)
    shape, dx = (16, 16, 16), 1.0 / 16
    # scale: the force of a unit mass on a particle four cells away
    scale = np.abs(_force(np.array([[0.5], [0.5], [0.5]]), np.array([1.0]),
                          np.array([[0.75], [0.5], [0.5]]), shape, dx)).max()
    assert scale > 0
    for _ in range(5):
        p = rng.uniform(0, 1, (3, 1))
        f = _force(p, np.array([1.0]), p, shape, dx)
        assert np.abs(f).max() <= 1e-12 * scale
    # two particles: equal and opposite forces, pulling toward each other
    p = np.array([[0.31, 0.52], [0.47, 0.58], [0.5, 0.44]])
    m = np.array([1.0, 2.5])
    f0 = _force(p[:, 1:], m[1:], p[:, :1], shape, dx)[:, 0] * m[0]
    f1 = _force(p[:, :1], m[:1], p[:, 1:], shape, dx)[:, 0] * m[1]
    assert np.allclose(f0, -f1, rtol=1e-10, atol=1e-12 * scale)
    assert np.dot(f0, p[:, 1] - p[:, 0]) > 0
