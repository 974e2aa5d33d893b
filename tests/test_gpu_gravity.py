"""The gravity input path through the C ABI (Sec. 2.4, Sec. 3.4) against the
oracle: the cloud-in-cell deposit (to the rounding of its atomic additions),
the multigrid Poisson solve against the exact solution of the discrete
7-point system within the bound its own residual gives, run-to-run bitwise
determinism, the fixed-cycle form equal to the tolerance form, the gas
density taken from a state, the centred gradient bitwise in the padded
layout (FP64 and FP32), and a gas step driven by that gravity equal to the
oracle's step bit for bit.  At 256^3 the solve meets its tolerance."""
import numpy as np
import pytest

import oracle
from gpu_harness import NG, aligned_ws, to_dev
from paper_1301_4498_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nyx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1301_4498_amd as nyx
    nyx.lib()
    return nyx


def _particles(rng, n, L):
    pos = rng.uniform(0, 1, (3, n)) * np.asarray(L)[:, None]
    # edge positions: on the boundary, just inside it, outside the domain
    pos[:, :4] = [[0.0, L[0] - 1e-12, -0.3 * L[0], 1.7 * L[0]],
                  [0.5 * L[1], 0.0, L[1], -1e-9],
                  [L[2] - 1e-13, 0.25 * L[2], 0.0, 2.2 * L[2]]]
    return pos, rng.uniform(0.5, 2.0, n)


def test_cic_deposit_matches_oracle(nyx):
    import torch
    rng = np.random.default_rng(11)
    shape, dx = (8, 12, 16), 1.0 / 16
    L = [16 * dx, 12 * dx, 8 * dx]
    pos, mass = _particles(rng, 20000, L)
    rho = torch.zeros(shape, dtype=torch.float64, device="cuda")
    nyx.cic_deposit(to_dev(pos), to_dev(mass), (16, 12, 8), dx, rho)
    got = rho.cpu().numpy()
    ref = oracle.cic_deposit(pos, mass, shape, dx)
    assert np.allclose(got, ref, rtol=1e-13, atol=0)
    assert abs(got.sum() * dx ** 3 - mass.sum()) <= 1e-12 * mass.sum()
    # accumulates into what is there
    nyx.cic_deposit(to_dev(pos[:, :10]), to_dev(mass[:10]), (16, 12, 8), dx, rho)
    ref2 = oracle.cic_deposit(pos[:, :10], mass[:10], shape, dx, rho=ref)
    assert np.allclose(rho.cpu().numpy(), ref2, rtol=1e-13, atol=0)



def test_cic_deposit_of_no_particles_is_a_no_op(nyx):
    import torch
    rho = torch.full((4, 6, 8), 1.5, dtype=torch.float64, device="cuda")
    empty = torch.zeros((3, 0), dtype=torch.float64, device="cuda")
    nyx.cic_deposit(empty, torch.zeros(0, dtype=torch.float64, device="cuda"), (8, 6, 4),
                    0.125, rho)
    torch.cuda.synchronize()
    assert torch.equal(rho, torch.full_like(rho, 1.5))

def _resid_ok(r, f, phi, dx, tol):
    """max|r| within tol max|f| plus the rounding of evaluating the 7-point
    residual in another order (terms of size 6 max|phi| / dx^2)."""
    slack = 2e-14 * (6.0 * np.abs(phi).max() / dx ** 2 + np.abs(f).max())
    return np.abs(r).max() <= tol * np.abs(f).max() + slack


def _lam_min(shape, dx):
    return min((2.0 - 2.0 * np.cos(2 * np.pi / n)) / dx ** 2 for n in shape)


@pytest.mark.parametrize("shape", [(32, 32, 32), (16, 24, 32), (12, 12, 12), (12, 20, 24)])
def test_poisson_solve_within_its_residual_bound(nyx, shape):
    import torch
    rng = np.random.default_rng(12)
    dx, coef = 1.0 / shape[2], 2.5
    rho = rng.lognormal(0.0, 0.6, shape)
    dom = (shape[2], shape[1], shape[0])
    solver = nyx.PoissonSolver(dom)
    phi = torch.zeros(shape, dtype=torch.float64, device="cuda")
    cyc, rel = solver.solve(to_dev(rho), phi, dx, coef, tol=1e-11, max_vcycles=40)
    print(shape, "V-cycles", cyc, "relative residual", rel, flush=True)
    got = phi.cpu().numpy()
    f = coef * (rho - rho.mean())
    r = f - oracle.laplacian7(got, dx)
    assert rel <= 1e-11 and _resid_ok(r, f, got, dx, 1e-11)
    assert cyc <= 40
    ref = oracle.poisson_solve(rho, dx, coef)
    err = np.sqrt(((got - ref) ** 2).sum())
    bound = np.sqrt((r ** 2).sum()) / _lam_min(shape, dx)
    assert err <= 1.01 * bound + 1e-13 * np.sqrt((ref ** 2).sum())
    assert abs(got.mean()) <= 1e-14 * np.abs(got).max()
    # the same inputs give the same bits; the fixed-cycle form equals it
    phi2 = torch.zeros_like(phi)
    solver.solve(to_dev(rho), phi2, dx, coef, tol=1e-11, max_vcycles=40)
    phi3 = torch.zeros_like(phi)
    solver.enqueue(to_dev(rho), phi3, dx, coef, cyc)
    assert torch.equal(phi, phi2) and torch.equal(phi, phi3)


def test_solve_with_gas_density_and_gradient_bitwise(nyx):
    import torch
    w = synth.config1(n=16, seed=13)
    rng = np.random.default_rng(13)
    shape, dx = (16, 16, 16), w.dx
    pos, mass = _particles(rng, 3000, [16 * dx] * 3)
    dom = (16, 16, 16)
    box = nyx.make_box((16, 16, 16), NG, dx)
    state = to_dev(w.state)
    rho = torch.zeros(shape, dtype=torch.float64, device="cuda")
    nyx.cic_deposit(to_dev(pos), to_dev(mass), dom, dx, rho)
    phi = torch.zeros(shape, dtype=torch.float64, device="cuda")
    solver = nyx.PoissonSolver(dom)
    coef = 4 * np.pi * 0.05 / w.a0
    cyc, rel = solver.solve(rho, phi, dx, coef, tol=1e-12, max_vcycles=40, state=state, box=box)
    assert rel <= 1e-12
    rho_t = rho.cpu().numpy() + w.state[0, NG:-NG, NG:-NG, NG:-NG]
    got = phi.cpu().numpy()
    f = coef * (rho_t - rho_t.mean())
    assert _resid_ok(f - oracle.laplacian7(got, dx), f, got, dx, 1e-12)
    # g = -grad(phi) in the padded layout, ghosts the periodic images
    g64 = torch.zeros((3,) + w.state.shape[1:], dtype=torch.float64, device="cuda")
    nyx.gravity_from_phi(phi, dom, dx, box, g64, nyx.NYX_FP64)
    ref = synth.pad_periodic(oracle.gradient(got, dx))
    assert np.array_equal(g64.cpu().numpy(), ref)
    g32 = torch.zeros((3,) + w.state.shape[1:], dtype=torch.float32, device="cuda")
    nyx.gravity_from_phi(phi, dom, dx, box, g32, nyx.NYX_MIXED)
    assert np.array_equal(g32.cpu().numpy(), ref.astype(np.float32))
    # a step driven by this gravity equals the oracle's step bit for bit
    prm = nyx.default_params()
    dt = oracle.estimate_dt(w.state, NG, w.a0, dx, 0.5)
    out = torch.empty_like(state)
    ws_n = nyx.workspace_bytes(prm, box)
    nyx.hydro_step(prm, box, state, g64, dt, w.a0, w.a_at(1), out, workspace=aligned_ws(ws_n))
    ref_out, _ = oracle.hydro_step(w.state, ref, NG, dt, dx, w.a0, w.a_at(1))
    v = (slice(None),) + (slice(NG, -NG),) * 3
    assert np.array_equal(out.cpu().numpy()[v], ref_out[v])


def test_poisson_256_meets_tolerance(nyx):
    import torch
    shape, dx = (256, 256, 256), 1.0 / 256
    print("poisson 256^3", flush=True)
    rng = np.random.default_rng(14)
    rho = synth.lognormal(rng, shape, 1.0, 0.5)
    solver = nyx.PoissonSolver((256, 256, 256))
    phi = torch.zeros(shape, dtype=torch.float64, device="cuda")
    cyc, rel = solver.solve(to_dev(rho), phi, dx, 1.0, tol=1e-10, max_vcycles=40)
    print("V-cycles", cyc, "relative residual", rel, flush=True)
    got = phi.cpu().numpy()
    f = rho - rho.mean()
    r = f - oracle.laplacian7(got, dx)
    assert rel <= 1e-10 and _resid_ok(r, f, got, dx, 1e-10)
    ref = oracle.poisson_solve(rho, dx, 1.0)
    err = np.sqrt(((got - ref) ** 2).sum())
    assert err <= 1.01 * np.sqrt((r ** 2).sum()) / _lam_min(shape, dx) + \
        1e-12 * np.sqrt((ref ** 2).sum())


def test_uniform_density_gives_zero_potential(nyx):
    import torch
    shape, dx = (16, 16, 16), 1.0 / 16
    solver = nyx.PoissonSolver((16, 16, 16))
    rho = torch.full(shape, 2.5, dtype=torch.float64, device="cuda")
    phi = torch.zeros(shape, dtype=torch.float64, device="cuda")
    cyc, rel = solver.solve(rho, phi, dx, 3.0, tol=1e-12, max_vcycles=40)
    assert cyc == 1 and rel == 0.0
    assert torch.count_nonzero(phi).item() == 0


def test_fixed_cycle_solve_and_gradient_replay_in_a_graph(nyx):
    """Fixed V-cycles (kernels only, warm-started from the previous phi) and
    the gradient, captured in one HIP graph: each replay equals the eager
    sequence bit for bit.  The deposit stays outside: its atomic additions
    may add in another order from run to run."""
    import torch
    rng = np.random.default_rng(15)
    shape, dx, dom = (32, 32, 32), 1.0 / 32, (32, 32, 32)
    rho = to_dev(synth.lognormal(rng, shape, 1.0, 0.4))
    box = nyx.make_box(dom, NG, dx)
    solver = nyx.PoissonSolver(dom)

    def run(phi, g):
        solver.enqueue(rho, phi, dx, 2.0, 3)
        nyx.gravity_from_phi(phi, dom, dx, box, g, nyx.NYX_MIXED)

    phi_e = torch.zeros(shape, dtype=torch.float64, device="cuda")
    g_e = torch.zeros((3, 40, 40, 40), dtype=torch.float32, device="cuda")
    eager = []
    for r in range(3):
        run(phi_e, g_e)
        torch.cuda.synchronize()
        eager.append((phi_e.cpu().numpy().copy(), g_e.cpu().numpy().copy()))
    phi_g = torch.zeros_like(phi_e)
    g_g = torch.zeros_like(g_e)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            run(phi_g, g_g)
    torch.cuda.synchronize()
    for r in range(3):
        graph.replay()
        torch.cuda.synchronize()
        _ = (rho * 1.0).sum().item()
        assert np.array_equal(phi_g.cpu().numpy(), eager[r][0]), r
        assert np.array_equal(g_g.cpu().numpy(), eager[r][1]), r
