"""Learned Riemann flux through the C ABI.

Bars: GPU FP32 loss and gradients equal the CPU FP64 backpropagation (whose
own pin is central differences) to 1e-4 relative; the BF16 MFMA inference
equals the FP64 forward pass to BF16 accuracy (2e-2 of the output scale);
with a zero residual tolerance every face falls back and the step is bitwise
the plain FP32-mixed step; harvested records are the two-shock solution of
their own states; a trained network keeps the density within 1e-3 relative L1
of the plain solver over 10 steps while reporting its fallback rate; what the
trained network gains over the solver without it is measured on the same
steps: the evaluations of the two-shock relations per face it saves (the
network's Newton step and residual check count as two) and the step times of
both, printed side by side (on this GPU the iterations it replaces are
cheaper than the network, so the learned step is slower); NaN weights fall
back on every face, bitwise the plain step."""
import numpy as np
import pytest

import oracle
from gpu_harness import NG, aligned_ws, to_dev
from paper_1301_4498_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1301_4498_amd as nyx
    from paper_1301_4498_amd import learn
    nyx.lib()
    return nyx, learn, torch


@pytest.fixture(scope="module")
def records(env):
    nyx, learn, torch = env
    ws = [synth.config2(n=48, seed=100 + s) for s in range(3)]
    rec = learn.harvest(ws, steps=4, keep_fraction=0.25, capacity=400000, seed=1)
    assert rec.shape[0] > 100000
    return rec


def test_harvest_records_are_solver_solutions(env, records):
    rec = records[:200].cpu().numpy().astype(np.float64)
    for r in rec:
        _, st, _ = oracle.riemann(r[:5], r[5:10])
        assert st["p"] == pytest.approx(r[10], rel=2e-6)
        assert st["rhoL"] == pytest.approx(r[12], rel=2e-6)
        assert st["rhoR"] == pytest.approx(r[13], rel=2e-6)
        assert abs(st["u"] - r[11]) <= 2e-6 * (abs(r[11]) + abs(r[1]) + abs(r[6]) + 1e-3)


def test_gradients_match_cpu_oracle(env, records):
    nyx, learn, torch = env
    f = learn.LearnedFlux(seed=5)
    sub = records[:512].contiguous()
    for it in range(3):
        loss, grad = f.loss_grad(sub)
        torch.cuda.synchronize()
        P = f.params.double().cpu().numpy()
        x, y = oracle.mlp_normalize(sub.double().cpu().numpy())
        lref, gref = oracle.mlp_loss_grad(P, x, y)
        g = grad.double().cpu().numpy()
        assert float(loss.item()) == pytest.approx(lref, rel=1e-4)
        assert np.linalg.norm(g - gref) <= 1e-4 * np.linalg.norm(gref), it
        f.adam(lr=1e-3)  # move away from the initial point and check again


def test_bf16_inference_matches_fp64_forward(env, records):
    nyx, learn, torch = env
    f = learn.LearnedFlux(seed=7)
    f.train(records[:100000].contiguous(), epochs=1, batch=4096)
    f.pack()
    sub = records[:4096].contiguous()
    out = f.predict(sub).double().cpu().numpy()
    P = f.params.double().cpu().numpy()
    x, _ = oracle.mlp_normalize(sub.double().cpu().numpy())
    ref = oracle.mlp_forward(P, x)
    scale = np.abs(ref).mean(axis=0) + 0.05
    err = np.abs(out - ref).mean(axis=0) / scale
    print("BF16 vs FP64 forward, mean abs error / scale per output:", err)
    assert err.max() <= 2e-2


def _run(nyx, torch, w, prm, steps, timing=None):
    """`steps` steps of one periodic box; with a list `timing`, the device
    milliseconds of the step loop are appended to it."""
    box = nyx.make_box(w.n, NG, w.dx)
    _, one = nyx.Batch.workspace_bytes(prm, [box])
    plan = nyx.Batch(prm, [box], aligned_ws(one))
    U = to_dev(w.state)
    V = torch.zeros_like(U)
    G = to_dev(w.grav, torch.float32)
    dts = torch.zeros(2, dtype=torch.float64, device="cuda")
    st = torch.zeros(10, dtype=torch.int64, device="cuda")
    plan.estimate_dt(U, w.a0, 0.5, dts[0:1])
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for k in range(steps):
        plan.step(U, G, dts[k % 2:k % 2 + 1], w.a_at(k), w.a_at(k + 1), V,
                  dt_next=dts[(k + 1) % 2:(k + 1) % 2 + 1], stats=st)
        plan.fill_ghosts(V)
        U, V = V, U
    e1.record()
    torch.cuda.synchronize()
    if timing is not None:
        timing.append(e0.elapsed_time(e1))
    return U.cpu().numpy(), nyx.stats_dict(st)


def test_zero_tolerance_falls_back_bitwise(env, records):
    nyx, learn, torch = env
    f = learn.LearnedFlux(seed=3)
    f.pack()
    w = synth.config2(n=32, seed=77)
    plain, st0 = _run(nyx, torch, w, nyx.default_params(precision=nyx.NYX_MIXED), 3)
    lp = learn.learned_params(f, tol=0.0, stages=7)
    got, st = _run(nyx, torch, w, lp, 3)
    assert np.array_equal(got, plain)
    assert st["mlp_used"] == 0
    assert st["mlp_fallback"] == st["riemann_calls"] == st0["riemann_calls"]


def test_nan_weights_fall_back_everywhere_bitwise(env, records):
    # a network whose weights are all NaN: every face must fall back, and
    # the step must be the plain FP32-mixed step bit for bit
    nyx, learn, torch = env
    f = learn.LearnedFlux(seed=3)
    f.params.fill_(float("nan"))
    f.pack()
    w = synth.config2(n=32, seed=78)
    plain, st0 = _run(nyx, torch, w, nyx.default_params(precision=nyx.NYX_MIXED), 3)
    got, st = _run(nyx, torch, w, learn.learned_params(f, tol=1e-3, stages=7), 3)
    assert np.array_equal(got, plain)
    assert st["mlp_used"] == 0
    assert st["mlp_fallback"] == st["riemann_calls"] == st0["riemann_calls"]
    assert st["nonfinite"] == 0


def test_trained_network_density_error_and_fallback(env, records):
    nyx, learn, torch = env
    f = learn.LearnedFlux(seed=11)
    hist = f.train(records.contiguous(), epochs=6, batch=8192)
    assert hist[-1] < hist[0]
    f.pack()
    w = synth.config2(n=48, seed=7)  # not a training seed
    plain, _ = _run(nyx, torch, w, nyx.default_params(precision=nyx.NYX_MIXED), 10)
    got, st = _run(nyx, torch, w, learn.learned_params(f, tol=1e-3, stages=7), 10)
    v, r = got[0, NG:-NG, NG:-NG, NG:-NG], plain[0, NG:-NG, NG:-NG, NG:-NG]
    l1 = np.abs(v - r).sum() / np.abs(r).sum()
    used, fb = st["mlp_used"], st["mlp_fallback"]
    print("loss history", hist)
    print("density L1 vs plain %.3e, network used on %d faces, fallback %d (%.1f%%)"
          % (l1, used, fb, 100.0 * fb / max(used + fb, 1)))
    assert used + fb == st["riemann_calls"]
    assert l1 <= 1e-3
    assert used > 0


def test_learned_gain_over_plain_solver(env, records):
    nyx, learn, torch = env
    f = learn.LearnedFlux(seed=13)
    f.train(records.contiguous(), epochs=6, batch=8192)
    f.pack()
    w = synth.config2(n=64, seed=7)
    res = {}
    for name, prm in (("plain", nyx.default_params(precision=nyx.NYX_MIXED)),
                      ("learned", learn.learned_params(f, tol=1e-3, stages=7))):
        _run(nyx, torch, w, prm, 1)  # warm-up
        ms = []
        U, st = _run(nyx, torch, w, prm, 5, timing=ms)
        res[name] = (U, st, ms[0])
    Up, sp, tp = res["plain"]
    Ul, sl, tl = res["learned"]
    v, r = Ul[0, NG:-NG, NG:-NG, NG:-NG], Up[0, NG:-NG, NG:-NG, NG:-NG]
    l1 = np.abs(v - r).sum() / np.abs(r).sum()
    # evaluations of the two-shock relations per face: the plain solver's
    # Newton iterations; for the learned form the network's Newton step and
    # residual check on every face plus the iterations of the faces that
    # fall back
    ep = sp["riemann_iters"] / sp["riemann_calls"]
    el = sl["riemann_iters"] / sl["riemann_calls"]
    fb = sl["mlp_fallback"] / max(sl["mlp_used"] + sl["mlp_fallback"], 1)
    print("two-shock evaluations per face: plain %.3f, learned %.3f (%.1f%% fewer; fallback "
          "%.2f%%); density L1 %.2e; 5 steps: plain %.2f ms, learned %.2f ms (%.2fx)"
          % (ep, el, 100.0 * (1 - el / ep), 100.0 * fb, l1, tp, tl, tp / tl))
    assert el < ep
    assert l1 <= 1e-3
