"""GPU parity of the HIP step against the FP64 oracle, through the C ABI.

Bar: FP64 build <= 1e-12 relative L1 per component after 10 steps (the two
evaluate the same expression trees without contraction, so bitwise equality
is expected and reported); the CFL reduction is exact, so dt must match
bitwise; counters must match exactly.  FP32-mixed build <= 1e-5 relative L1
after 10 steps.  Both sides are fed the oracle's dt sequence."""
import numpy as np
import pytest

import oracle
from gpu_harness import NG, gpu_run, oracle_run, rel_l1, to_dev, aligned_ws
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


@pytest.fixture(scope="module")
def cfg1_oracle():
    w = synth.config1()
    a_list = [w.a_at(k) for k in range(w.steps + 1)]
    U, dts, stats = oracle_run(w.state, w.grav, w.dx, a_list)
    # the CFL step of the final state, for the fused dt_next check
    return w, a_list, U, dts, stats


def test_estimate_dt_bitwise(nyx):
    import torch
    for seed, n in ((1, (32, 32, 32)), (5, (10, 6, 14)), (9, (2, 4, 2))):
        U, _ = synth.random_box(n, seed=seed, a=0.5)
        box = nyx.make_box(n, NG, 1.0 / 32)
        prm = nyx.default_params()
        d = torch.zeros(1, dtype=torch.float64, device="cuda")
        ws = aligned_ws(256)
        nyx.estimate_dt(prm, box, to_dev(U), 0.5, 0.5, d, ws)
        torch.cuda.synchronize()
        want = oracle.estimate_dt(U, NG, 0.5, 1.0 / 32, 0.5)
        assert d.item() == want, (n, d.item(), want)


def test_fp64_step_matches_oracle_config1(nyx, cfg1_oracle):
    w, a_list, U_ref, dts, st_ref = cfg1_oracle
    prm = nyx.default_params()
    U, dt_next, st = gpu_run(w.state, w.grav, w.n, w.dx, a_list, dts, prm)
    errs = rel_l1(U, U_ref)
    print("fp64 rel L1 per component:", errs)
    print("max abs diff:", np.abs(U - U_ref)[:, NG:-NG, NG:-NG, NG:-NG].max())
    assert max(errs) <= 1e-12
    # fused CFL of each new state equals the oracle's next dt (exact max)
    assert dt_next[:-1] == dts[1:]
    # device counters equal the oracle's
    for k in range(len(st)):
        for key, v in st_ref[k].items():
            assert st[k][key] == v, (k, key, st[k][key], v)


def test_fp64_step_bitwise_config1(nyx, cfg1_oracle):
    w, a_list, U_ref, dts, _ = cfg1_oracle
    U, _, _ = gpu_run(w.state, w.grav, w.n, w.dx, a_list, dts, nyx.default_params())
    v = U[:, NG:-NG, NG:-NG, NG:-NG]
    r = U_ref[:, NG:-NG, NG:-NG, NG:-NG]
    assert np.array_equal(v, r), "FP64 build is not bitwise equal to the oracle"


def test_mixed_step_config1(nyx, cfg1_oracle):
    w, a_list, U_ref, dts, _ = cfg1_oracle
    prm = nyx.default_params(precision=nyx.NYX_MIXED)
    U, _, st = gpu_run(w.state, w.grav, w.n, w.dx, a_list, dts, prm)
    errs = rel_l1(U, U_ref)
    print("mixed rel L1 per component:", errs)
    assert max(errs) <= 1e-5
    assert all(s["nonfinite"] == 0 for s in st)


@pytest.mark.parametrize("n", [(10, 6, 14), (2, 2, 2), (18, 4, 8)])
def test_fp64_ragged_and_minimum_boxes(nyx, n):
    U0, g = synth.random_box(n, seed=sum(n), a=0.5)
    a_list = [0.5, 0.5025, 0.505]
    dx = 1.0 / 16
    U_ref, dts, _ = oracle_run(U0, g, dx, a_list)
    U, _, _ = gpu_run(U0, g, n, dx, a_list, dts, nyx.default_params())
    assert max(rel_l1(U, U_ref)) <= 1e-12


def test_fp64_strided_layout_and_wider_ghosts(nyx):
    # state at a nonzero offset, padded component stride, ng = 5
    import torch
    n, ng = (8, 10, 6), 5
    rng = np.random.default_rng(3)
    shape = (n[2], n[1], n[0])
    rho = synth.lognormal(rng, shape, 1.0, 0.5)
    u = rng.normal(0, 0.3, (3,) + shape)
    p = synth.lognormal(rng, shape, 0.6, 0.3)
    U0 = synth.pad_periodic(synth.conserved(rho, u, p, 0.5), ng)
    g0 = synth.pad_periodic(rng.normal(0, 0.05, (3,) + shape), ng)
    dt = 2e-3
    Uo_ref, st_ref = oracle.hydro_step(U0, g0, ng, dt, 1 / 8, 0.5, 0.501)
    P = U0[0].size
    off, stride = 1000, P + 77
    flat = np.zeros(off + 6 * stride)
    for c in range(6):
        flat[off + c * stride: off + c * stride + P] = U0[c].ravel()
    gflat = np.zeros(3 * (P + 13) + 40)
    for c in range(3):
        gflat[40 + c * (P + 13): 40 + c * (P + 13) + P] = g0[c].ravel()
    box = nyx.make_box(n, ng, 1 / 8, state_off=off, grav_off=40, comp_stride=stride,
                       grav_stride=P + 13)
    prm = nyx.default_params()
    Ui = to_dev(flat)
    Uo = torch.zeros_like(Ui)
    ws = aligned_ws(nyx.workspace_bytes(prm, box))
    nyx.hydro_step(prm, box, Ui, to_dev(gflat), dt, 0.5, 0.501, Uo, workspace=ws)
    torch.cuda.synchronize()
    out = Uo.cpu().numpy()
    got = np.stack([out[off + c * stride: off + c * stride + P].reshape(U0.shape[1:]) for c in range(6)])
    assert np.array_equal(got[:, ng:-ng, ng:-ng, ng:-ng], Uo_ref[:, ng:-ng, ng:-ng, ng:-ng])
    # ghost cells of the output are not written
    assert np.all(got[:, :ng] == 0)


def test_degenerate_states(nyx):
    # uniform state, gas at rest, and a cold hypersonic flow that takes the
    # E-from-e branch of the dual-energy sync everywhere
    n = (8, 8, 8)
    shape = (8, 8, 8)
    cases = []
    for rho, u, p in ((1.0, (0.0, 0.0, 0.0), 1.0), (0.5, (3.0, -2.0, 1.0), 0.2),
                      (1.0, (100.0, 0.0, 0.0), 1e-3)):
        U = synth.pad_periodic(synth.conserved(np.full(shape, rho),
                                               np.stack([np.full(shape, x) for x in u]),
                                               np.full(shape, p), 1.0))
        cases.append(U)
    g = np.zeros((3,) + cases[0].shape[1:])
    for U0 in cases:
        a_list = [1.0, 1.0]
        U_ref, dts, st_ref = oracle_run(U0, g, 1 / 8, a_list)
        U, _, st = gpu_run(U0, g, n, 1 / 8, a_list, dts, nyx.default_params())
        assert np.array_equal(U[:, NG:-NG, NG:-NG, NG:-NG], U_ref[:, NG:-NG, NG:-NG, NG:-NG])
        assert st[0] == {**st_ref[0], "mlp_used": 0, "mlp_fallback": 0}


def test_floor_and_negative_density_are_counted(nyx):
    # a cell with negative density and one with negative internal energy in
    # the input: floors are applied and counted, nothing is clamped silently
    U0, g = synth.random_box((8, 8, 8), seed=31, a=0.5)
    U0[0, NG + 3, NG + 3, NG + 3] = -0.1
    U0[5, NG + 5, NG + 2, NG + 6] = -1e-3
    a_list = [0.5, 0.5]
    U_ref, dts, st_ref = oracle_run(U0, g, 1 / 8, a_list, dts=[1e-3])
    U, _, st = gpu_run(U0, g, (8, 8, 8), 1 / 8, a_list, dts, nyx.default_params())
    assert st_ref[0]["floor_hits"] > 0
    for key, v in st_ref[0].items():
        assert st[0][key] == v, key
    assert np.array_equal(U[:, NG:-NG, NG:-NG, NG:-NG], U_ref[:, NG:-NG, NG:-NG, NG:-NG],
                          equal_nan=True)
