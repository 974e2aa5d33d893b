"""Parity at the full sizes of the level, the smooth 256^3 box over its step
count, and the learned flux on a fresh 256^3 box, each in the launch
configuration bench.py times (batched plans, device-resident dt, autotuned
launch orders).

Launch orders and (where bench.py chooses one) the launch mode come from the
plan's autotuners, as in bench.py, and every plan reads the ghost cells from
their periodic images inside the step, as bench.py does: the inputs' ghost
cells are NaN here, and after the steps exactly those values are still NaN
(no ghost cell read into a valid one, none written).

  * 4096-box level (edges from {16, 24, 32, 48, 64}): FP64 for 2 steps with
    per-box dt, then FP32-mixed with that dt sequence; 20 sampled boxes (4
    per x-edge length, every other edge random) against the oracle box by
    box.  FP64 bitwise; FP32-mixed <= 1e-5 relative L1 per component.
  * 256^3 smooth box, 10 steps: FP64 with its fused dt, then FP32-mixed with
    that dt sequence.  The oracle runs windows of 8^3 valid cells with a
    40-cell halo: a step's result in a cell depends only on data within 4
    cells, so after k steps the window's inner region shrinks by 4 cells per
    side and step, and the 8^3 centre after 10 steps is exact.  FP64
    bitwise; FP32-mixed <= 1e-5 relative L1.
  * learned flux on a fresh-seed 256^3 box of the same type, 20 steps: the
    density stays within 1e-3 relative L1 of the plain FP32-mixed step; the
    fallback rate is printed.
"""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from gpu_harness import NG, aligned_ws, to_dev
from paper_1301_4498_amd import synth

pytestmark = pytest.mark.gpu

EDGES = (16, 24, 32, 48, 64)


@pytest.fixture(scope="module")
def nyx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1301_4498_amd as nyx
    nyx.lib()
    return nyx


def _threads():
    import os
    return max(1, min(16, len(os.sched_getaffinity(0))))


def _poison_ghosts(buf, shapes, soffs):
    """NaN into every ghost cell of the boxes (shapes n, state offsets) of a
    flat state buffer; returns how many values were set."""
    nan, count = float("nan"), 0
    for n, so in zip(shapes, soffs):
        px, py, pz = (n[0] + 2 * NG, n[1] + 2 * NG, n[2] + 2 * NG)
        v = buf[so:so + 6 * px * py * pz].view(6, pz, py, px)
        for sl in ((slice(None), slice(None, NG)), (slice(None), slice(-NG, None)),
                   (slice(None), slice(None), slice(None, NG)), (slice(None), slice(None), slice(-NG, None)),
                   (slice(None), slice(None), slice(None), slice(None, NG)),
                   (slice(None), slice(None), slice(None), slice(-NG, None))):
            v[sl] = nan
        count += 6 * (px * py * pz - n[0] * n[1] * n[2])
    return count


def test_level4096_sampled_boxes_against_oracle(nyx):
    import torch
    shapes = synth.config3_shapes()
    state, grav, offs = synth.level_fields_torch(shapes)
    boxes = [nyx.make_box(n, NG, 1.0 / 256, state_off=so, grav_off=go)
             for n, (so, go) in zip(shapes, offs)]
    steps, a0, a1 = 2, 0.25, 0.255
    a = [a0 + (a1 - a0) * k / 10 for k in range(steps + 1)]
    # 4 boxes per x-edge length
    pick = []
    for e in EDGES:
        pick += [b for b, n in enumerate(shapes) if n[0] == e][:4]
    assert len(pick) == 20

    def host_box(t, b, ncomp):
        n = shapes[b]
        P = (n[0] + 8) * (n[1] + 8) * (n[2] + 8)
        off = offs[b][0] if ncomp == 6 else offs[b][1]
        return t[off:off + ncomp * P].double().cpu().numpy().reshape(ncomp, n[2] + 8, n[1] + 8,
                                                                    n[0] + 8)

    U0 = {b: host_box(state, b, 6) for b in pick}
    G0 = {b: host_box(grav, b, 3) for b in pick}
    results = {}
    dt_seq = torch.zeros((steps + 1, len(boxes)), dtype=torch.float64, device="cuda")
    for prec in ("fp64", "mixed"):
        prm = nyx.default_params(precision=nyx.NYX_FP64 if prec == "fp64" else nyx.NYX_MIXED)
        G = grav if prec == "fp64" else grav.float()
        _, one = nyx.Batch.workspace_bytes(prm, boxes)
        # as bench.py sizes it: one group when it fits beside the buffers
        free = torch.cuda.mem_get_info()[0]
        wsb = min(one, int(free - 3 * state.numel() * 8 - (8 << 30)))
        plan = nyx.Batch(prm, boxes, aligned_ws(wsb))
        if prec == "mixed":
            assert plan.num_groups == 1
        # as bench.py steps it: every box its own periodic domain, the ghost
        # cells read from their images inside the step (here NaN in both
        # buffers, and never written)
        plan.set_ghost_source(0)
        bufs = [state.clone(), state.clone()]
        nghost = _poison_ghosts(bufs[0], shapes, [o[0] for o in offs])
        _poison_ghosts(bufs[1], shapes, [o[0] for o in offs])
        if prec == "fp64":
            plan.estimate_dt(bufs[0], a[0], 0.5, dt_seq[0])
        plan.autotune(bufs[0], G, dt_seq[0], a[0], a[1], bufs[1], reps=1)
        if prec == "mixed":
            # the launch mode bench.py times (staged, persistent or fused)
            plan.autotune_mode(bufs[0], G, dt_seq[0], a[0], a[1], bufs[1], reps=1)
        print("level4096 %s: %d boxes in %d group(s), tuning %s, launch mode %d"
              % (prec, len(boxes), plan.num_groups, plan.tuning(), plan.launch_mode), flush=True)
        for k in range(steps):
            plan.step(bufs[k % 2], G, dt_seq[k], a[k], a[k + 1], bufs[(k + 1) % 2],
                      dt_next=dt_seq[k + 1] if prec == "fp64" else None)
        torch.cuda.synchronize()
        fin = bufs[steps % 2]
        assert int(torch.isnan(fin).sum().item()) == nghost
        assert int((~torch.isfinite(fin)).sum().item()) == nghost
        results[prec] = {b: host_box(fin, b, 6) for b in pick}
        plan.close()
        del plan, bufs, G, fin  # the plan object holds its workspace
        torch.cuda.empty_cache()
    dts = dt_seq.cpu().numpy()

    def ref(b):
        U = U0[b].copy()
        for k in range(steps):
            dk = float(dts[k, b])
            if k == 0:
                assert dk == oracle.estimate_dt(U, NG, a[0], 1.0 / 256, 0.5)
            U, _ = oracle.hydro_step(U, G0[b], NG, dk, 1.0 / 256, a[k], a[k + 1])
            synth.fill_periodic_inplace(U)
        return b, U

    with ThreadPoolExecutor(max_workers=_threads()) as ex:
        refs = dict(ex.map(ref, pick))
    worst = 0.0
    for b in pick:
        r = refs[b][:, NG:-NG, NG:-NG, NG:-NG]
        g64 = results["fp64"][b][:, NG:-NG, NG:-NG, NG:-NG]
        assert np.array_equal(g64, r), (b, shapes[b])
        gm = results["mixed"][b][:, NG:-NG, NG:-NG, NG:-NG]
        rel = (np.abs(gm - r).sum(axis=(1, 2, 3)) / np.abs(r).sum(axis=(1, 2, 3))).max()
        worst = max(worst, rel)
    print("level4096: 20 sampled boxes, FP64 bitwise, FP32-mixed worst relative L1 %.2e" % worst)
    assert worst <= 1e-5


def _periodic_window(f, lo, size):
    """f: padded periodic (ncomp, N+8, N+8, N+8); the region of valid-index
    origin lo (x, y, z) and edge `size`, wrapping around the domain."""
    N = f.shape[-1] - 2 * NG
    v = f[:, NG:-NG, NG:-NG, NG:-NG]
    idx = [(np.arange(size) + lo[d]) % N for d in range(3)]
    return np.ascontiguousarray(v[:, idx[2]][:, :, idx[1]][:, :, :, idx[0]])


def test_box256_ten_steps_windows(nyx):
    import torch
    w = synth.config2(n=256)
    steps = 10
    H = 4 * steps
    Wn = 8
    a = [w.a_at(k) for k in range(steps + 1)]
    box = nyx.make_box(w.n, NG, w.dx)
    out = {}
    dts = torch.zeros(steps + 1, dtype=torch.float64, device="cuda")
    for prec in ("fp64", "mixed"):
        p = nyx.default_params(precision=nyx.NYX_FP64 if prec == "fp64" else nyx.NYX_MIXED)
        _, one = nyx.Batch.workspace_bytes(p, [box])
        plan = nyx.Batch(p, [box], aligned_ws(one))
        # as bench.py steps it: ghost cells read from their periodic images
        # inside the step (here NaN, and never written)
        plan.set_ghost_source(0)
        U = [to_dev(w.state), None]
        U[1] = U[0].clone()
        nghost = _poison_ghosts(U[0].view(-1), [w.n], [0])
        _poison_ghosts(U[1].view(-1), [w.n], [0])
        G = to_dev(w.grav, torch.float64 if prec == "fp64" else torch.float32)
        if prec == "fp64":
            plan.estimate_dt(U[0], w.a0, 0.5, dts[0:1])
        plan.autotune(U[0], G, dts[0:1], a[0], a[1], U[1], reps=1)
        plan.autotune_mode(U[0], G, dts[0:1], a[0], a[1], U[1], reps=1)
        print("box256 %s: tuning %s, launch mode %d" % (prec, plan.tuning(), plan.launch_mode),
              flush=True)
        for k in range(steps):
            plan.step(U[k % 2], G, dts[k:k + 1], a[k], a[k + 1], U[(k + 1) % 2],
                      dt_next=dts[k + 1:k + 2] if prec == "fp64" else None)
        torch.cuda.synchronize()
        out[prec] = U[steps % 2].cpu().numpy()
        assert int(np.isnan(out[prec]).sum()) == nghost
        plan.close()
        del U, G
    dtl = dts.cpu().tolist()
    corners = [(0, 0, 0), (124, 250, 61), (253, 96, 200)]

    def ref(lo):
        # window origin (valid index) of the 8^3 target, halo H, wrapped
        lo_h = [lo[d] - H for d in range(3)]
        U = _periodic_window(w.state, lo_h, Wn + 2 * H)
        G = _periodic_window(w.grav, lo_h, Wn + 2 * H)
        for k in range(steps):
            U, _ = oracle.hydro_step(U, G, NG, dtl[k], w.dx, a[k], a[k + 1])
            # the outer 4 layers are now stale: the valid cells become the
            # next step's padded box
            U = np.ascontiguousarray(U[:, NG:-NG, NG:-NG, NG:-NG])
            G = np.ascontiguousarray(G[:, NG:-NG, NG:-NG, NG:-NG])
        return lo, U

    with ThreadPoolExecutor(max_workers=min(_threads(), len(corners))) as ex:
        refs = dict(ex.map(ref, corners))
    worst = 0.0
    for lo in corners:
        r = refs[lo]
        assert r.shape[1:] == (Wn, Wn, Wn)
        for prec in ("fp64", "mixed"):
            g = _periodic_window(out[prec], lo, Wn)
            if prec == "fp64":
                assert np.array_equal(g, r), lo
            else:
                rel = (np.abs(g - r).sum(axis=(1, 2, 3)) / np.abs(r).sum(axis=(1, 2, 3))).max()
                worst = max(worst, rel)
    print("box256 x 10 steps, 3 windows: FP64 bitwise, FP32-mixed worst relative L1 %.2e" % worst)
    assert worst <= 1e-5


def test_learned_flux_fresh_256_box_twenty_steps(nyx):
    import torch
    from paper_1301_4498_amd import learn
    ws = [synth.config2(n=64, seed=100 + s) for s in range(4)]
    rec = learn.harvest(ws, steps=8, keep_fraction=0.31, capacity=12_000_000, seed=100)
    f = learn.LearnedFlux(seed=1)
    hist = f.train(rec, epochs=3, batch=16384)
    f.pack()
    del rec
    w = synth.config2(n=256, seed=7)
    box = nyx.make_box(w.n, NG, w.dx)
    res = {}
    for name, prm in (("mixed", nyx.default_params(precision=nyx.NYX_MIXED)),
                      ("learned", learn.learned_params(f, tol=1e-3, stages=7))):
        _, one = nyx.Batch.workspace_bytes(prm, [box])
        plan = nyx.Batch(prm, [box], aligned_ws(one))
        plan.set_ghost_source(0)  # as bench.py steps it
        U = [to_dev(w.state), None]
        U[1] = U[0].clone()
        _poison_ghosts(U[0].view(-1), [w.n], [0])
        _poison_ghosts(U[1].view(-1), [w.n], [0])
        G = to_dev(w.grav, torch.float32)
        dts = torch.zeros(2, dtype=torch.float64, device="cuda")
        st = torch.zeros(10, dtype=torch.int64, device="cuda")
        plan.estimate_dt(U[0], w.a0, 0.5, dts[0:1])
        for k in range(w.steps):
            plan.step(U[k % 2], G, dts[k % 2:k % 2 + 1], w.a_at(k), w.a_at(k + 1),
                      U[(k + 1) % 2], dt_next=dts[(k + 1) % 2:(k + 1) % 2 + 1], stats=st)
        torch.cuda.synchronize()
        res[name] = (U[w.steps % 2][0, NG:-NG, NG:-NG, NG:-NG].cpu().numpy(), nyx.stats_dict(st))
        plan.close()
    (rm, _), (rl, sl) = res["mixed"], res["learned"]
    l1 = np.abs(rl - rm).sum() / np.abs(rm).sum()
    fb = sl["mlp_fallback"] / max(sl["mlp_used"] + sl["mlp_fallback"], 1)
    print("learned flux, 256^3 seed 7, 20 steps: density L1 vs plain mixed %.2e, fallback "
          "%.3f%%, loss %s" % (l1, 100 * fb, hist))
    assert np.isfinite(rl).all()
    assert l1 <= 1e-3
    assert sl["mlp_used"] > 0
