"""The persistent launch mode of batched plans (NYX_LAUNCH_PERSISTENT: the
seven stages of a group in one launch, work items from atomic queues, grid
barriers between stages) against the staged launches through the C ABI.
Every item runs the staged kernel's code, so the new state, the next dt and
the counters must be equal bit for bit: on uneven boxes in one and in
several groups, in FP64 (also against the oracle), FP32-mixed and with the
learned flux, on the 4096-box level, and replayed from a captured HIP graph.
No launch may end at the barrier's time limit."""
import numpy as np
import pytest

import oracle
from gpu_harness import NG, aligned_ws, to_dev
from paper_1301_4498_amd import synth

pytestmark = pytest.mark.gpu

SHAPES = [(16, 24, 32), (48, 16, 16), (24, 24, 24), (64, 16, 32), (32, 48, 16), (16, 16, 16)]


@pytest.fixture(scope="module")
def nyx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1301_4498_amd as nyx
    nyx.lib()
    return nyx


def _pack(nyx, shapes, seed0=3000, a=0.25, dx=1 / 256):
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


def _steps(nyx, torch, plan, Ui, G, dt, a_list, mode, stats=True):
    """len(a_list) - 1 steps in `mode` from Ui; returns (state, dt list, stats)."""
    plan.set_launch_mode(mode)
    assert plan.launch_mode == mode
    U = [Ui.clone(), torch.empty_like(Ui)]
    dts = [dt.clone()]
    st = torch.zeros(10, dtype=torch.int64, device="cuda")
    for k in range(len(a_list) - 1):
        dn = torch.zeros_like(dt)
        plan.step(U[k % 2], G, dts[-1], a_list[k], a_list[k + 1], U[(k + 1) % 2], dt_next=dn,
                  stats=st if stats else None)
        plan.fill_ghosts(U[(k + 1) % 2])
        dts.append(dn)
    torch.cuda.synchronize()
    assert not plan.persistent_aborted()
    return U[(len(a_list) - 1) % 2], [d.cpu().numpy() for d in dts], nyx.stats_dict(st)


@pytest.mark.parametrize("form", ["fp64", "mixed", "learned"])
@pytest.mark.parametrize("ws_mode", ["one_group", "min"])
def test_persistent_equals_staged(nyx, form, ws_mode):
    import torch
    from paper_1301_4498_amd import learn
    if form == "fp64":
        prm = nyx.default_params()
    elif form == "mixed":
        prm = nyx.default_params(precision=nyx.NYX_MIXED)
    else:
        f = learn.LearnedFlux(seed=9)
        f.pack()
        prm = learn.learned_params(f, tol=1e-3, stages=7)
        prm._keep = f
    boxes, states, gravs, flat, gflat = _pack(nyx, SHAPES)
    mn, one = nyx.Batch.workspace_bytes(prm, boxes)
    plan = nyx.Batch(prm, boxes, aligned_ws(one if ws_mode == "one_group" else mn))
    assert (plan.num_groups == 1) == (ws_mode == "one_group")
    Ui = to_dev(flat)
    G = to_dev(gflat, torch.float64 if form == "fp64" else torch.float32)
    dt = torch.zeros(len(boxes), dtype=torch.float64, device="cuda")
    plan.estimate_dt(Ui, 0.25, 0.5, dt)
    a_list = [0.25, 0.2505, 0.251]
    print("persistent vs staged: %s, %d group(s)" % (form, plan.num_groups), flush=True)
    s_state, s_dts, s_st = _steps(nyx, torch, plan, Ui, G, dt, a_list, nyx.NYX_LAUNCH_STAGED)
    p_state, p_dts, p_st = _steps(nyx, torch, plan, Ui, G, dt, a_list, nyx.NYX_LAUNCH_PERSISTENT)
    assert torch.equal(s_state, p_state)
    for a, b in zip(s_dts, p_dts):
        assert np.array_equal(a, b)
    assert s_st == p_st
    assert s_st["riemann_calls"] > 0
    if form == "fp64":
        # and box by box equal to the oracle after the two steps
        got = p_state.cpu().numpy()
        for b, (U, g, bx) in enumerate(zip(states, gravs, boxes)):
            ref = U.copy()
            for k in range(2):
                ref, _ = oracle.hydro_step(ref, g, NG, float(s_dts[k][b]), 1 / 256, a_list[k],
                                           a_list[k + 1])
                synth.fill_periodic_inplace(ref)
            out = got[bx.state_off:bx.state_off + U.size].reshape(U.shape)
            assert np.array_equal(out[:, NG:-NG, NG:-NG, NG:-NG], ref[:, NG:-NG, NG:-NG, NG:-NG])
    plan.close()


def test_persistent_level4096_equals_staged(nyx):
    import torch
    shapes = synth.config3_shapes()
    state, grav, offs = synth.level_fields_torch(shapes, grav_dtype=torch.float32)
    boxes = [nyx.make_box(n, NG, 1.0 / 256, state_off=so, grav_off=go)
             for n, (so, go) in zip(shapes, offs)]
    prm = nyx.default_params(precision=nyx.NYX_MIXED)
    _, one = nyx.Batch.workspace_bytes(prm, boxes)
    plan = nyx.Batch(prm, boxes, aligned_ws(one))
    dt = torch.zeros(len(boxes), dtype=torch.float64, device="cuda")
    plan.estimate_dt(state, 0.25, 0.5, dt)
    print("persistent level4096: %d boxes, %d group(s)" % (len(boxes), plan.num_groups), flush=True)
    s_state, s_dts, s_st = _steps(nyx, torch, plan, state, grav, dt, [0.25, 0.2505],
                                  nyx.NYX_LAUNCH_STAGED)
    s_state = s_state.clone()
    p_state, p_dts, p_st = _steps(nyx, torch, plan, state, grav, dt, [0.25, 0.2505],
                                  nyx.NYX_LAUNCH_PERSISTENT)
    assert torch.equal(s_state, p_state)
    assert np.array_equal(s_dts[1], p_dts[1])
    assert s_st == p_st
    mode, ms = plan.autotune_mode(state, grav, dt, 0.25, 0.2505, p_state, reps=2)
    print("level4096 mixed step: staged %.3f ms, persistent %.3f ms, fused %.3f ms, kept mode %d"
          % (ms[0], ms[1], ms[2], mode))
    assert mode in (nyx.NYX_LAUNCH_STAGED, nyx.NYX_LAUNCH_PERSISTENT, nyx.NYX_LAUNCH_FUSED)
    assert min(ms) > 0
    plan.close()


def test_persistent_graph_replay(nyx):
    import torch
    prm = nyx.default_params(precision=nyx.NYX_MIXED)
    boxes, states, gravs, flat, gflat = _pack(nyx, SHAPES)
    _, one = nyx.Batch.workspace_bytes(prm, boxes)
    plan = nyx.Batch(prm, boxes, aligned_ws(one))
    plan.set_launch_mode(nyx.NYX_LAUNCH_PERSISTENT)
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

    # eager reference: two steps from Ui
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
    assert not plan.persistent_aborted()
    plan.close()
