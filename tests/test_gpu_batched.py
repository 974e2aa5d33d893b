"""Batched plans through the C ABI: many uneven boxes in shared buffers.

Bar: FP64 batched results are bitwise equal to the oracle box by box (the
same arithmetic as a single-box launch), independent of how boxes are grouped;
per-box CFL steps are bitwise; ghost fills equal numpy's periodic copies; a
captured HIP graph replays to the same state as eager launches; every launch
order the autotuner can pick gives the same bits, and its cached choice is
reapplied without timing."""
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


def _pack(nyx, shapes, seed0=3000, a=0.25, dx=1 / 256):
    """Boxes of the batched level in one state and one gravity buffer."""
    boxes, states, gravs = [], [], []
    soff = goff = 0
    for b, n in enumerate(shapes):
        U, g = synth.config3_box(seed0 - 3000 + b, n, a) if seed0 == 3000 else synth.random_box(n, seed0 + b, a)
        P = U[0].size
        boxes.append(nyx.make_box(n, NG, dx, state_off=soff, grav_off=goff))
        states.append(U)
        gravs.append(g)
        soff += 6 * P
        goff += 3 * P
    flat = np.concatenate([u.ravel() for u in states])
    gflat = np.concatenate([g.ravel() for g in gravs])
    return boxes, states, gravs, flat, gflat


def _unpack(flat, states, boxes):
    out = []
    for U, bx in zip(states, boxes):
        out.append(flat[bx.state_off: bx.state_off + U.size].reshape(U.shape))
    return out


SHAPES = [(16, 24, 32), (48, 16, 16), (24, 24, 24), (64, 16, 32), (32, 48, 16), (16, 16, 16)]


@pytest.mark.parametrize("ws_mode", ["one_group", "min"])
def test_batched_fp64_equals_oracle_per_box(nyx, ws_mode):
    import torch
    prm = nyx.default_params()
    boxes, states, gravs, flat, gflat = _pack(nyx, SHAPES)
    mn, one = nyx.Batch.workspace_bytes(prm, boxes)
    ws = aligned_ws(one if ws_mode == "one_group" else mn)
    plan = nyx.Batch(prm, boxes, ws)
    if ws_mode == "min":
        assert plan.num_groups > 1
    else:
        assert plan.num_groups == 1
    Ui = to_dev(flat)
    Uo = torch.zeros_like(Ui)
    G = to_dev(gflat)
    dt = torch.zeros(len(boxes), dtype=torch.float64, device="cuda")
    dtn = torch.zeros_like(dt)
    st = torch.zeros(10, dtype=torch.int64, device="cuda")
    plan.estimate_dt(Ui, 0.25, 0.5, dt)
    plan.step(Ui, G, dt, 0.25, 0.2505, Uo, dt_next=dtn, stats=st)
    torch.cuda.synchronize()
    got = _unpack(Uo.cpu().numpy(), states, boxes)
    dts = dt.cpu().numpy()
    dtns = dtn.cpu().numpy()
    calls = 0
    for b, (U, g, bx) in enumerate(zip(states, gravs, boxes)):
        want_dt = oracle.estimate_dt(U, NG, 0.25, 1 / 256, 0.5)
        assert dts[b] == want_dt
        ref, s = oracle.hydro_step(U, g, NG, want_dt, 1 / 256, 0.25, 0.2505)
        calls += s["riemann_calls"]
        assert np.array_equal(got[b][:, NG:-NG, NG:-NG, NG:-NG], ref[:, NG:-NG, NG:-NG, NG:-NG]), b
        synth.fill_periodic_inplace(ref)
        assert dtns[b] == oracle.estimate_dt(ref, NG, 0.2505, 1 / 256, 0.5)
    assert nyx.stats_dict(st)["riemann_calls"] == calls
    plan.min_dt(dt)
    torch.cuda.synchronize()
    assert np.all(dt.cpu().numpy() == dts.min())
    plan.close()


def test_batched_mixed_close_to_oracle(nyx):
    import torch
    prm = nyx.default_params(precision=nyx.NYX_MIXED)
    boxes, states, gravs, flat, gflat = _pack(nyx, SHAPES[:4])
    _, one = nyx.Batch.workspace_bytes(prm, boxes)
    plan = nyx.Batch(prm, boxes, aligned_ws(one))
    Ui = to_dev(flat)
    Uo = torch.zeros_like(Ui)
    dt = torch.zeros(len(boxes), dtype=torch.float64, device="cuda")
    plan.estimate_dt(Ui, 0.25, 0.5, dt)
    plan.step(Ui, to_dev(gflat, torch.float32), dt, 0.25, 0.2505, Uo)
    torch.cuda.synchronize()
    got = _unpack(Uo.cpu().numpy(), states, boxes)
    for b, (U, g) in enumerate(zip(states, gravs)):
        ref, _ = oracle.hydro_step(U, g, NG, float(dt[b].item()), 1 / 256, 0.25, 0.2505)
        v, r = got[b][:, NG:-NG, NG:-NG, NG:-NG], ref[:, NG:-NG, NG:-NG, NG:-NG]
        for c in range(6):
            assert np.abs(v[c] - r[c]).sum() / np.abs(r[c]).sum() <= 1e-5


def test_ghost_fills(nyx):
    import torch
    prm = nyx.default_params()
    # mode 0: every box is its own periodic domain
    boxes, states, gravs, flat, gflat = _pack(nyx, SHAPES[:3])
    mn, _ = nyx.Batch.workspace_bytes(prm, boxes)
    plan = nyx.Batch(prm, boxes, aligned_ws(mn))
    junk = flat.copy()
    for U, bx in zip(states, boxes):
        v = junk[bx.state_off: bx.state_off + U.size].reshape(U.shape)
        v[:, :NG] = -7.0
        v[:, :, -NG:] = -7.0
        v[:, :, :, :NG] = -7.0
    T = to_dev(junk)
    plan.fill_ghosts(T, mode=0)
    torch.cuda.synchronize()
    assert np.array_equal(T.cpu().numpy(), flat)
    # mode 1: a 2 x 3 x 2 grid of 8^3 boxes tiling one periodic domain
    gx, gy, gz, m = 2, 3, 2, 8
    rng = np.random.default_rng(4)
    dom = rng.normal(size=(6, gz * m, gy * m, gx * m))
    pad = synth.pad_periodic(dom)
    bl, parts = [], []
    off = 0
    for bz in range(gz):
        for by in range(gy):
            for bx in range(gx):
                part = pad[:, bz * m: bz * m + m + 2 * NG, by * m: by * m + m + 2 * NG,
                           bx * m: bx * m + m + 2 * NG].copy()
                bl.append(nyx.make_box((m, m, m), NG, 1 / 16, state_off=off))
                parts.append(part)
                off += part.size
    want = np.concatenate([p.ravel() for p in parts])
    zeroed = []
    for p in parts:
        q = np.zeros_like(p)
        q[:, NG:-NG, NG:-NG, NG:-NG] = p[:, NG:-NG, NG:-NG, NG:-NG]
        zeroed.append(q)
    T = to_dev(np.concatenate([q.ravel() for q in zeroed]))
    mn, _ = nyx.Batch.workspace_bytes(prm, bl)
    plan2 = nyx.Batch(prm, bl, aligned_ws(mn))
    plan2.fill_ghosts(T, mode=1, grid=(gx, gy, gz))
    torch.cuda.synchronize()
    assert np.array_equal(T.cpu().numpy(), want)


def test_ghost_fill_tiled_odd_layouts(nyx):
    """Mode 1 on boxes that are not cubes, with ghost width 5, state offsets
    that are multiples of nothing and a different component stride in every
    box (a source box's stride is its own): every ghost cell equals the
    periodic domain's, the valid cells and the padding between components
    are untouched."""
    import torch
    prm = nyx.default_params()
    gx, gy, gz, n, ng = 3, 2, 2, (10, 6, 8), 5
    rng = np.random.default_rng(41)
    dom = rng.normal(size=(6, gz * n[2], gy * n[1], gx * n[0]))
    pad = synth.pad_periodic(dom, ng)
    bl, want, start = [], [], []
    off = 13
    for bz in range(gz):
        for by in range(gy):
            for bx in range(gx):
                part = pad[:, bz * n[2]: bz * n[2] + n[2] + 2 * ng, by * n[1]: by * n[1] + n[1] + 2 * ng,
                           bx * n[0]: bx * n[0] + n[0] + 2 * ng]
                P = part[0].size
                cs = P + 7 * len(bl) + 3
                bl.append(nyx.make_box(n, ng, 1 / 16, state_off=off, comp_stride=cs))
                want.append(part)
                start.append((off, cs))
                off += 6 * cs + 11
    flat = np.full(off, np.nan)
    full = np.full(off, np.nan)
    for (o, cs), part in zip(start, want):
        for c in range(6):
            z = np.zeros_like(part[c])
            z[ng:-ng, ng:-ng, ng:-ng] = part[c][ng:-ng, ng:-ng, ng:-ng]
            flat[o + c * cs: o + c * cs + z.size] = z.ravel()
            full[o + c * cs: o + c * cs + z.size] = part[c].ravel()
    T = to_dev(flat)
    mn, _ = nyx.Batch.workspace_bytes(prm, bl)
    plan = nyx.Batch(prm, bl, aligned_ws(mn))
    plan.fill_ghosts(T, mode=1, grid=(gx, gy, gz))
    torch.cuda.synchronize()
    got = T.cpu().numpy()
    assert np.array_equal(got, full, equal_nan=True)
    plan.close()


@pytest.mark.parametrize("tune", [0, 13])
def test_graph_replay_matches_eager(nyx, tune):
    # capture [step with fused dt_next -> ghost fill] x 2 into a HIP graph and
    # replay it; every replay must reproduce the eager sequence bitwise (with
    # the default launch order and with a tuned one: cell-major rows, slab
    # pencils of 32 rows)
    import torch
    prm = nyx.default_params()
    boxes, states, gravs, flat, gflat = _pack(nyx, SHAPES[:3])
    _, one = nyx.Batch.workspace_bytes(prm, boxes)
    plan = nyx.Batch(prm, boxes, aligned_ws(one))
    plan.set_tuning([tune] * 7)
    G = to_dev(gflat)
    nb = len(boxes)

    def run(A, B, dts, a0):
        plan.step(A, G, dts[0], a0, a0 + 1e-4, B, dt_next=dts[1])
        plan.fill_ghosts(B)
        plan.step(B, G, dts[1], a0 + 1e-4, a0 + 2e-4, A, dt_next=dts[0])
        plan.fill_ghosts(A)

    # eager reference: 3 rounds of 2 steps
    A = to_dev(flat)
    B = torch.zeros_like(A)
    dts = [torch.zeros(nb, dtype=torch.float64, device="cuda") for _ in range(2)]
    plan.estimate_dt(A, 0.25, 0.5, dts[0])
    eager = []
    for r in range(3):
        run(A, B, dts, 0.25)
        torch.cuda.synchronize()
        eager.append(A.cpu().numpy().copy())
    # graph
    A2 = to_dev(flat)
    B2 = torch.zeros_like(A2)
    d2 = [torch.zeros(nb, dtype=torch.float64, device="cuda") for _ in range(2)]
    plan.estimate_dt(A2, 0.25, 0.5, d2[0])
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            run(A2, B2, d2, 0.25)
    torch.cuda.synchronize()
    for r in range(3):
        g.replay()
        torch.cuda.synchronize()
        _ = (A2 * 1.0).sum().item()  # unrelated eager work between replays
        assert np.array_equal(A2.cpu().numpy(), eager[r]), r


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_every_launch_order_gives_the_same_bits(nyx, prec, tmp_path):
    import torch
    p = nyx.default_params(precision=nyx.NYX_FP64 if prec == "fp64" else nyx.NYX_MIXED)
    boxes, states, gravs, flat, gflat = _pack(nyx, SHAPES)
    mn, one = nyx.Batch.workspace_bytes(p, boxes)
    plan = nyx.Batch(p, boxes, aligned_ws(mn))  # several groups
    assert plan.num_groups > 1
    Ui = to_dev(flat)
    G = to_dev(gflat, torch.float64 if prec == "fp64" else torch.float32)
    dt = torch.zeros(len(boxes), dtype=torch.float64, device="cuda")
    plan.estimate_dt(Ui, 0.25, 0.5, dt)
    outs = []
    for c in range(16):
        plan.set_tuning([c] * 7)
        assert plan.tuning() == [c] * 7
        Uo = torch.zeros_like(Ui)
        dn = torch.zeros_like(dt)
        plan.step(Ui, G, dt, 0.25, 0.2505, Uo, dt_next=dn)
        torch.cuda.synchronize()
        outs.append((Uo.cpu().numpy(), dn.cpu().numpy()))
    for U, dn in outs[1:]:
        assert np.array_equal(U, outs[0][0])
        assert np.array_equal(dn, outs[0][1])
    # the autotuner keeps one candidate per stage, reports its timings and
    # writes the same result as a step
    cache = str(tmp_path / "tune.json")
    Uo = torch.zeros_like(Ui)
    dn = torch.zeros_like(dt)
    tune, ms = plan.autotune(Ui, G, dt, 0.25, 0.2505, Uo, dt_next=dn, reps=2, cache=cache)
    torch.cuda.synchronize()
    assert np.array_equal(dn.cpu().numpy(), outs[0][1])
    print(prec, "tuning", tune, "ms per stage and candidate", ms)
    assert len(tune) == 7 and all(0 <= t < 16 for t in tune)
    assert plan.tuning() == tune
    assert all(ms[i][tune[i]] == min(ms[i]) for i in range(7))
    assert np.array_equal(Uo.cpu().numpy(), outs[0][0])
    # a second plan over the same boxes takes the cached choice
    plan2 = nyx.Batch(p, boxes, aligned_ws(mn))
    tune2, ms2 = plan2.autotune(Ui, G, dt, 0.25, 0.2505, Uo, cache=cache)
    assert ms2 is None and tune2 == tune and plan2.tuning() == tune
    plan.close()
    plan2.close()


def _periodic_parts(grid, n, ng, seed, a):
    """A periodic domain of gx*gy*gz boxes of n cells (box order x fastest):
    each box's padded state and gravity with its ghosts taken from the domain.
    Smooth flow plus per-cell noise, so a ghost read from a wrong cell shows."""
    gx, gy, gz = grid
    NX, NY, NZ = gx * n[0], gy * n[1], gz * n[2]
    rng = np.random.default_rng(seed)
    z, y, x = np.meshgrid(np.arange(NZ) / NZ, np.arange(NY) / NY, np.arange(NX) / NX, indexing="ij")
    tw = 2 * np.pi
    rho = 1.0 + 0.3 * np.sin(tw * (x + 2 * y)) * np.cos(tw * z) + 0.05 * rng.random(x.shape)
    u = np.stack([0.4 * np.sin(tw * (y + z)), 0.3 * np.cos(tw * (x + z)), -0.2 * np.sin(tw * (x - y))])
    u = u + 0.02 * rng.normal(size=u.shape)
    p = 0.6 + 0.2 * np.cos(tw * (x + y + z)) + 0.05 * rng.random(x.shape)
    pad = synth.pad_periodic(synth.conserved(rho, u, p, a), ng)
    gpad = synth.pad_periodic(0.01 * rng.normal(size=(3, NZ, NY, NX)), ng)
    parts = []
    for bz in range(gz):
        for by in range(gy):
            for bx in range(gx):
                sl = (slice(None), slice(bz * n[2], bz * n[2] + n[2] + 2 * ng),
                      slice(by * n[1], by * n[1] + n[1] + 2 * ng), slice(bx * n[0], bx * n[0] + n[0] + 2 * ng))
                parts.append((n, pad[sl].copy(), gpad[sl].copy()))
    return parts


def _lay_out(nyx, parts, ng, dx):
    """Boxes at odd offsets with a different component stride each; the state
    with every ghost cell NaN, the same with the ghosts filled, the gravity."""
    boxes, spans = [], []
    off = goff = 0
    for b, (n, U, g) in enumerate(parts):
        P = U[0].size
        cs = P + 7 * b + 3
        boxes.append(nyx.make_box(n, ng, dx, state_off=off + 5, grav_off=goff, comp_stride=cs))
        spans.append((off + 5, cs))
        off += 6 * cs + 11
        goff += 3 * P
    bare = np.zeros(off)
    full = np.zeros(off)
    for (o, cs), (n, U, g) in zip(spans, parts):
        for c in range(6):
            v = np.full(U[c].shape, np.nan)
            v[ng:-ng, ng:-ng, ng:-ng] = U[c][ng:-ng, ng:-ng, ng:-ng]
            bare[o + c * cs: o + c * cs + U[c].size] = v.ravel()
            full[o + c * cs: o + c * cs + U[c].size] = U[c].ravel()
    gflat = np.concatenate([g.ravel() for _, _, g in parts])
    return boxes, spans, bare, full, gflat


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("case", ["tiled", "tiled_ng_eq_n", "own_periodic"])
def test_step_takes_ghosts_from_their_sources(nyx, prec, case):
    """A plan told where the input's ghost cells come from (each box periodic,
    or the neighbouring box of a tiling grid) never reads them: stepping an
    input whose ghosts are NaN gives, in every launch mode, the bits of
    stepping it after the same-level ghost fill, leaves the input as it was,
    and in FP64 equals the oracle box by box."""
    import torch
    a0, a1, dx = 0.25, 0.2505, 1 / 64
    if case == "tiled":
        grid, mode, parts = (3, 2, 2), 1, _periodic_parts((3, 2, 2), (10, 6, 8), NG, 71, a0)
    elif case == "tiled_ng_eq_n":
        grid, mode, parts = (2, 2, 2), 1, _periodic_parts((2, 2, 2), (4, 4, 4), NG, 72, a0)
    else:
        grid, mode = (1, 1, 1), 0
        parts = [p for s, n in enumerate(SHAPES[:4]) for p in _periodic_parts((1, 1, 1), n, NG, 80 + s, a0)]
    prm = nyx.default_params(precision=nyx.NYX_FP64 if prec == "fp64" else nyx.NYX_MIXED)
    boxes, spans, bare, full, gflat = _lay_out(nyx, parts, NG, dx)
    _, one = nyx.Batch.workspace_bytes(prm, boxes)
    plan = nyx.Batch(prm, boxes, aligned_ws(one))
    G = to_dev(gflat, torch.float64 if prec == "fp64" else torch.float32)
    filled = to_dev(bare)
    plan.fill_ghosts(filled, mode=mode, grid=grid)
    torch.cuda.synchronize()
    assert np.array_equal(filled.cpu().numpy(), full)
    dt = torch.zeros(len(boxes), dtype=torch.float64, device="cuda")
    plan.estimate_dt(filled, a0, 0.5, dt)
    Ui = to_dev(bare)
    outs = {}
    for lm in (nyx.NYX_LAUNCH_STAGED, nyx.NYX_LAUNCH_FUSED, nyx.NYX_LAUNCH_PERSISTENT):
        plan.set_launch_mode(lm)
        ref = torch.zeros_like(Ui)
        got = torch.zeros_like(Ui)
        plan.set_ghost_source(-1)
        plan.step(filled, G, dt, a0, a1, ref)
        plan.set_ghost_source(mode, grid)
        plan.step(Ui, G, dt, a0, a1, got)
        plan.set_ghost_source(-1)
        torch.cuda.synchronize()
        r, g = ref.cpu().numpy(), got.cpu().numpy()
        assert np.isfinite(r).all()
        assert np.array_equal(r, g), lm
        outs[lm] = g
    assert np.array_equal(Ui.cpu().numpy(), bare, equal_nan=True)
    if prec == "fp64":
        dts = dt.cpu().numpy()
        got = outs[nyx.NYX_LAUNCH_STAGED]
        for b, ((o, cs), (n, U, gr)) in enumerate(zip(spans, parts)):
            want, _ = oracle.hydro_step(U, gr, NG, float(dts[b]), dx, a0, a1)
            v = np.stack([got[o + c * cs: o + c * cs + U[c].size].reshape(U[c].shape) for c in range(6)])
            assert np.array_equal(v[:, NG:-NG, NG:-NG, NG:-NG], want[:, NG:-NG, NG:-NG, NG:-NG]), b
    plan.close()


def test_set_ghost_source_rejects_bad_shapes(nyx):
    prm = nyx.default_params()
    boxes = [nyx.make_box((8, 8, 8), NG, 1 / 16, state_off=6 * 16 ** 3 * b, grav_off=3 * 16 ** 3 * b)
             for b in range(4)]
    _, one = nyx.Batch.workspace_bytes(prm, boxes)
    plan = nyx.Batch(prm, boxes, aligned_ws(one))
    for mode, grid in ((1, (2, 2, 2)), (1, (4, 1, 0)), (1, (3, 1, 1))):
        with pytest.raises(nyx.NyxError):
            plan.set_ghost_source(mode, grid)
    for mode in (-2, 2):
        with pytest.raises(nyx.NyxError):
            plan.set_ghost_source(mode, (1, 1, 1))
    plan.set_ghost_source(1, (4, 1, 1))
    plan.set_ghost_source(1, (1, 2, 2))
    plan.set_ghost_source(0)
    plan.set_ghost_source(-1)
    plan.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_ghost_source_in_a_captured_graph(nyx, prec):
    """Two chained steps that take the ghosts from their sources (the input of
    the second step has never had its ghosts filled), captured once in a HIP
    graph with the fused dt_next: every replay equals the eager sequence bit
    for bit, and no ghost cell of either buffer is ever written."""
    import torch
    prm = nyx.default_params(precision=nyx.NYX_FP64 if prec == "fp64" else nyx.NYX_MIXED)
    grid = (3, 2, 2)
    parts = _periodic_parts(grid, (10, 6, 8), NG, 73, 0.25)
    boxes, spans, bare, full, gflat = _lay_out(nyx, parts, NG, 1 / 64)
    _, one = nyx.Batch.workspace_bytes(prm, boxes)
    plan = nyx.Batch(prm, boxes, aligned_ws(one))
    plan.set_launch_mode(nyx.NYX_LAUNCH_FUSED)
    plan.set_ghost_source(1, grid)
    G = to_dev(gflat, torch.float64 if prec == "fp64" else torch.float32)
    nb = len(boxes)

    def run(A, B, dts, a0):
        plan.step(A, G, dts[0], a0, a0 + 1e-4, B, dt_next=dts[1])
        plan.step(B, G, dts[1], a0 + 1e-4, a0 + 2e-4, A, dt_next=dts[0])

    def start():
        A = to_dev(bare)
        B = to_dev(np.full(bare.shape, np.nan))
        dts = [torch.zeros(nb, dtype=torch.float64, device="cuda") for _ in range(2)]
        plan.estimate_dt(A, 0.25, 0.5, dts[0])
        return A, B, dts

    A, B, dts = start()
    eager = []
    for r in range(3):
        run(A, B, dts, 0.25)
        torch.cuda.synchronize()
        eager.append(A.cpu().numpy().copy())
    ghosts = np.isnan(bare)
    for e in eager:
        assert np.isnan(e[ghosts]).all() and np.isfinite(e[~ghosts]).all()
    A2, B2, d2 = start()
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            run(A2, B2, d2, 0.25)
    torch.cuda.synchronize()
    for r in range(3):
        g.replay()
        torch.cuda.synchronize()
        _ = (G * 1.0).sum().item()  # unrelated eager work between replays
        assert np.array_equal(A2.cpu().numpy(), eager[r], equal_nan=True), r
    plan.close()
