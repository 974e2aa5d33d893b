"""The fused final stage of batched plans (NYX_LAUNCH_FUSED: the final
Riemann solves and the conservative update as one launch of column tiles
marching in z, the final face states kept in LDS and registers) against the
staged launches through the C ABI.  Every face and cell runs the staged
kernels' code, so the new state, the next dt and the counters must be equal
bit for bit: on boxes whose tiles are partial in x and in y, narrow boxes (2
cells across), boxes cut into several z chunks, several groups, in FP64
(also against the oracle) and in FP32-mixed, replayed from a captured HIP
graph, and on the 512^3 stress domain as 512 patches of 64^3."""
import numpy as np
import pytest

import oracle
from gpu_harness import NG, aligned_ws, to_dev
from paper_1301_4498_amd import synth

pytestmark = pytest.mark.gpu

# tiles are TX = min(nx, 64) by TY = min(ny, 512 / TX) columns over chunks of
# at most 64 planes: partial in x (80, 130), partial in y (20 rows of 8, 48
# rows of 32, 24 rows of 21), boxes 2 cells across in x or y, and boxes
# taller than one chunk (130 = 64 + 64 + 2 planes)
SHAPES = [(16, 24, 32), (80, 20, 8), (130, 10, 6), (24, 24, 24), (16, 48, 8), (2, 6, 4),
          (6, 2, 4), (64, 64, 16), (10, 8, 130)]


@pytest.fixture(scope="module")
def nyx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1301_4498_amd as nyx
    nyx.lib()
    return nyx


def _pack(nyx, shapes, a=0.25, dx=1 / 256):
    boxes, states, gravs = [], [], []
    soff = goff = 0
    for b, n in enumerate(shapes):
        U, g = synth.config3_box(b, n, a)
        P = U[0].size
        boxes.append(nyx.make_box(n, NG, dx, state_off=soff, grav_off=goff))
        states.append(U)
        gravs.append(g)
        soff += 6 * P
        goff += 3 * P
    return boxes, states, gravs, np.concatenate([u.ravel() for u in states]), \
        np.concatenate([g.ravel() for g in gravs])


def _steps(nyx, torch, plan, Ui, G, dt, a_list, mode):
    """len(a_list) - 1 steps in `mode` from Ui; returns (state, dt list, stats)."""
    plan.set_launch_mode(mode)
    assert plan.launch_mode == mode
    U = [Ui.clone(), torch.empty_like(Ui)]
    dts = [dt.clone()]
    st = torch.zeros(10, dtype=torch.int64, device="cuda")
    for k in range(len(a_list) - 1):
        dn = torch.zeros_like(dt)
        plan.step(U[k % 2], G, dts[-1], a_list[k], a_list[k + 1], U[(k + 1) % 2], dt_next=dn,
                  stats=st)
        plan.fill_ghosts(U[(k + 1) % 2])
        dts.append(dn)
    torch.cuda.synchronize()
    return U[(len(a_list) - 1) % 2], [d.cpu().numpy() for d in dts], nyx.stats_dict(st)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("ws_mode", ["one_group", "min"])
def test_fused_equals_staged(nyx, prec, ws_mode):
    import torch
    prm = nyx.default_params(precision=nyx.NYX_FP64 if prec == "fp64" else nyx.NYX_MIXED)
    boxes, states, gravs, flat, gflat = _pack(nyx, SHAPES)
    mn, one = nyx.Batch.workspace_bytes(prm, boxes)
    plan = nyx.Batch(prm, boxes, aligned_ws(one if ws_mode == "one_group" else mn))
    assert (plan.num_groups == 1) == (ws_mode == "one_group")
    Ui = to_dev(flat)
    G = to_dev(gflat, torch.float64 if prec == "fp64" else torch.float32)
    dt = torch.zeros(len(boxes), dtype=torch.float64, device="cuda")
    plan.estimate_dt(Ui, 0.25, 0.5, dt)
    a_list = [0.25, 0.2505, 0.251]
    print("fused vs staged: %s, %d group(s)" % (prec, plan.num_groups), flush=True)
    s_state, s_dts, s_st = _steps(nyx, torch, plan, Ui, G, dt, a_list, nyx.NYX_LAUNCH_STAGED)
    f_state, f_dts, f_st = _steps(nyx, torch, plan, Ui, G, dt, a_list, nyx.NYX_LAUNCH_FUSED)
    assert torch.equal(s_state, f_state)
    for a, b in zip(s_dts, f_dts):
        assert np.array_equal(a, b)
    assert s_st == f_st
    assert s_st["riemann_calls"] > 0
    if prec == "fp64":
        # box by box equal to the oracle after the two steps
        got = f_state.cpu().numpy()
        for b, (U, g, bx) in enumerate(zip(states, gravs, boxes)):
            ref = U.copy()
            for k in range(2):
                ref, _ = oracle.hydro_step(ref, g, NG, float(s_dts[k][b]), 1 / 256, a_list[k],
                                           a_list[k + 1])
                synth.fill_periodic_inplace(ref)
            out = got[bx.state_off:bx.state_off + U.size].reshape(U.shape)
            assert np.array_equal(out[:, NG:-NG, NG:-NG, NG:-NG], ref[:, NG:-NG, NG:-NG, NG:-NG]), \
                (b, SHAPES[b])
    plan.close()


def test_fused_graph_replay(nyx):
    import torch
    prm = nyx.default_params(precision=nyx.NYX_MIXED)
    boxes, states, gravs, flat, gflat = _pack(nyx, SHAPES)
    _, one = nyx.Batch.workspace_bytes(prm, boxes)
    plan = nyx.Batch(prm, boxes, aligned_ws(one))
    plan.set_launch_mode(nyx.NYX_LAUNCH_FUSED)
    Ui = to_dev(flat)
    G = to_dev(gflat, torch.float32)
    dt = torch.zeros(len(boxes), dtype=torch.float64, device="cuda")
    plan.estimate_dt(Ui, 0.25, 0.5, dt)
    bufs = [Ui.clone(), torch.empty_like(Ui)]
    dts = [dt.clone(), torch.zeros_like(dt)]

    def two_steps():
        for k in range(2):
            plan.step(bufs[k], G, dts[k], 0.25, 0.2505, bufs[1 - k], dt_next=dts[1 - k])
            plan.fill_ghosts(bufs[1 - k])

    two_steps()
    torch.cuda.synchronize()
    want = bufs[0].clone()
    want_dt = dts[0].clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            two_steps()
    torch.cuda.synchronize()
    for rep in range(3):
        bufs[0].copy_(Ui)
        dts[0].copy_(dt)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        _ = (bufs[1] * 2.0).sum().item()  # unrelated eager work between replays
        assert torch.equal(bufs[0], want), rep
        assert torch.equal(dts[0], want_dt), rep
    plan.close()


def test_fused_stress_patches_equal_staged(nyx):
    """The headline configuration: the 512^3 stress domain as 512 patches of
    64^3 in one FP32-mixed plan, two steps with the patch-grid ghost fill."""
    import torch
    n, m = 512, 64
    grid = (n // m,) * 3
    state, grav = synth.stress_fields_torch(n=n)
    A0 = torch.cat([p.reshape(-1) for p in synth.split_patches(state, grid)])
    G32 = torch.cat([p.reshape(-1).float() for p in synth.split_patches(grav, grid)])
    del state, grav
    P = (m + 2 * NG) ** 3
    boxes = [nyx.make_box((m, m, m), NG, 1.0 / n, state_off=6 * P * b, grav_off=3 * P * b)
             for b in range(grid[0] * grid[1] * grid[2])]
    prm = nyx.default_params(precision=nyx.NYX_MIXED)
    _, one = nyx.Batch.workspace_bytes(prm, boxes)
    plan = nyx.Batch(prm, boxes, aligned_ws(one))
    assert plan.num_groups == 1
    dt = torch.zeros(len(boxes), dtype=torch.float64, device="cuda")
    plan.estimate_dt(A0, 0.10, 0.5, dt)
    nyx_min = dt.min()
    dt.fill_(float(nyx_min))
    res = {}
    for mode in (nyx.NYX_LAUNCH_STAGED, nyx.NYX_LAUNCH_FUSED):
        plan.set_launch_mode(mode)
        U = [A0.clone(), torch.empty_like(A0)]
        st = torch.zeros(10, dtype=torch.int64, device="cuda")
        dn = torch.zeros_like(dt)
        for k in range(2):
            plan.step(U[k], G32, dt, 0.10 + 0.001 * k, 0.101 + 0.001 * k, U[1 - k],
                      dt_next=dn if k == 1 else None, stats=st)
            plan.fill_ghosts(U[1 - k], mode=1, grid=grid)
        torch.cuda.synchronize()
        res[mode] = (U[0], dn.clone(), nyx.stats_dict(st))
        print("stress patches, mode %d: stats %s" % (mode, res[mode][2]), flush=True)
        del U
    (s_state, s_dn, s_st), (f_state, f_dn, f_st) = res[nyx.NYX_LAUNCH_STAGED], \
        res[nyx.NYX_LAUNCH_FUSED]
    assert bool(torch.isfinite(f_state).all())
    assert torch.equal(s_state, f_state)
    assert torch.equal(s_dn, f_dn)
    assert s_st == f_st
    plan.close()


VARIANTS = {"plm": dict(recon=1), "linear": dict(riemann=2), "gravity_form2": dict(grav_energy_form=2),
            "all_three": dict(recon=1, riemann=2, grav_energy_form=2), "gamma14_expansion": dict(gamma=1.4)}


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("variant", sorted(VARIANTS))
def test_fused_equals_staged_variants(nyx, prec, variant):
    """The scheme variants of Sec. 3.2 (PLM, the linearised solver, energy
    gravity form 2, all three, gamma = 1.4 with the expansion term) through
    the fused final stage: bitwise the staged launches."""
    import torch
    prm = nyx.default_params(precision=nyx.NYX_FP64 if prec == "fp64" else nyx.NYX_MIXED,
                             **VARIANTS[variant])
    shapes = SHAPES[:4]
    boxes, states, gravs, flat, gflat = _pack(nyx, shapes)
    _, one = nyx.Batch.workspace_bytes(prm, boxes)
    plan = nyx.Batch(prm, boxes, aligned_ws(one))
    Ui = to_dev(flat)
    G = to_dev(gflat, torch.float64 if prec == "fp64" else torch.float32)
    dt = torch.zeros(len(boxes), dtype=torch.float64, device="cuda")
    plan.estimate_dt(Ui, 0.25, 0.5, dt)
    a_list = [0.25, 0.2505, 0.251]
    s_state, s_dts, s_st = _steps(nyx, torch, plan, Ui, G, dt, a_list, nyx.NYX_LAUNCH_STAGED)
    f_state, f_dts, f_st = _steps(nyx, torch, plan, Ui, G, dt, a_list, nyx.NYX_LAUNCH_FUSED)
    assert torch.equal(s_state, f_state)
    for a, b in zip(s_dts, f_dts):
        assert np.array_equal(a, b)
    assert s_st == f_st
    plan.close()


@pytest.mark.parametrize("stages", [3, 4, 7])
def test_fused_with_learned_flux(nyx, stages):
    """The learned flux on stages 0-1 (the x front stays staged, the fused
    final stage runs the plain solver), on the final stage only (the x front
    is fused, the final stage stays staged) and on all three (both staged):
    the fused mode gives the staged launches' bits, counters included."""
    import torch
    from paper_1301_4498_amd import learn
    f = learn.LearnedFlux(seed=9)
    f.pack()
    prm = learn.learned_params(f, tol=1e-3, stages=stages)
    boxes, states, gravs, flat, gflat = _pack(nyx, SHAPES[:4])
    _, one = nyx.Batch.workspace_bytes(prm, boxes)
    plan = nyx.Batch(prm, boxes, aligned_ws(one))
    Ui = to_dev(flat)
    G = to_dev(gflat, torch.float32)
    dt = torch.zeros(len(boxes), dtype=torch.float64, device="cuda")
    plan.estimate_dt(Ui, 0.25, 0.5, dt)
    a_list = [0.25, 0.2505, 0.251]
    s_state, s_dts, s_st = _steps(nyx, torch, plan, Ui, G, dt, a_list, nyx.NYX_LAUNCH_STAGED)
    f_state, f_dts, f_st = _steps(nyx, torch, plan, Ui, G, dt, a_list, nyx.NYX_LAUNCH_FUSED)
    assert torch.equal(s_state, f_state)
    for a, b in zip(s_dts, f_dts):
        assert np.array_equal(a, b)
    assert s_st == f_st
    assert s_st["mlp_used"] + s_st["mlp_fallback"] > 0
    plan.close()
