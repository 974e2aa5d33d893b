"""Two-level synchronisation through the C ABI (Sec. 4.3: flux registers fed
by the batched steps, nyx_reflux, nyx_average_down) against the oracle.  One
coarse step of eight 8^3 boxes and two fine substeps of three fine boxes
(with a fine-fine face and neighbours across the periodic boundary), fine
ghosts filled from the coarse level interpolated in time.  FP64:
the synchronised coarse level and the fine level equal the oracle's bit for
bit, with the plan split into one or several workspace groups; FP32-mixed:
within 1e-5 relative L1, and its composite sums conserved."""
import numpy as np
import pytest

import oracle
from gpu_harness import NG, aligned_ws, to_dev
from paper_1301_4498_amd import synth
from test_oracle_sync import advance_two_levels, composite_sums, two_level_setup

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
def reference():
    cboxes, cdatas, fboxes, fdatas, cdom, dom = two_level_setup()
    cnew, fnew, cflux, ffl, dt_c, dt_f, stats = advance_two_levels(cboxes, cdatas, fboxes,
                                                                   fdatas, cdom, dom)
    csync = [x.copy() for x in cnew]
    nf, nc = oracle.reflux_average_down(cboxes, NG, 1.0 / cdom[0], csync, cflux, dt_c, fboxes,
                                        NG, dom, fnew, ffl, dt_f)
    return dict(setup=(cboxes, cdatas, fboxes, fdatas, cdom, dom), csync=csync, fnew=fnew,
                dt_c=dt_c, nfaces=nf, ncov=nc)


def _pack(nyx, layout, arrays, dx):
    boxes, soff, goff = [], 0, 0
    for (n, _), a in zip(layout, arrays):
        P = a[0].size
        boxes.append(nyx.make_box(n, NG, dx, state_off=soff, grav_off=goff))
        soff += 6 * P
        goff += 3 * P
    return boxes, np.concatenate([a.ravel() for a in arrays]), goff


def _unpack(flat, arrays):
    out, off = [], 0
    for a in arrays:
        out.append(flat[off:off + a.size].reshape(a.shape))
        off += a.size
    return out


def _gpu_two_levels(nyx, prm, setup, dt_c, groups, a0=0.5, a1=0.505, mode=None):
    import torch
    cboxes, cdatas, fboxes, fdatas, cdom, dom = setup
    clo = [lo for _, lo in cboxes]
    flo = [lo for _, lo in fboxes]
    cb, cflat, cg = _pack(nyx, cboxes, cdatas, 1.0 / cdom[0])
    fb, fflat, fg = _pack(nyx, fboxes, fdatas, 1.0 / dom[0])
    gdt = torch.float64 if prm.precision == nyx.NYX_FP64 else torch.float32
    cstate, fstate = to_dev(cflat), to_dev(fflat)
    cgrav = torch.zeros(cg, dtype=gdt, device="cuda")
    fgrav = torch.zeros(fg, dtype=gdt, device="cuda")
    cfill = nyx.FillPlan(cb, clo, cdom)
    ffill = nyx.FillPlan(fb, flo, dom, coarse=(cb, clo))
    sync = nyx.SyncPlan((fb, flo), (cb, clo), dom)
    reg = sync.register()

    def batch(boxes):
        mn, one = nyx.Batch.workspace_bytes(prm, boxes)
        b = nyx.Batch(prm, boxes, aligned_ws(mn if groups else one))
        assert (b.num_groups > 1) == groups
        return b

    cbat, fbat = batch(cb), batch(fb)
    if mode is not None:
        cbat.set_launch_mode(mode)
        fbat.set_launch_mode(mode)
    cbat.set_flux_register(sync, 0, reg)
    fbat.set_flux_register(sync, 1, reg)
    dtc = torch.full((len(cb),), dt_c, dtype=torch.float64, device="cuda")
    dtf = torch.full((len(fb),), 0.5 * dt_c, dtype=torch.float64, device="cuda")
    am = 0.5 * (a0 + a1)
    cfill.fill(cstate)
    cnew = cstate.clone()
    cbat.step(cstate, cgrav, dtc, a0, a1, cnew)
    cfill.fill(cnew)
    ffill.fill(fstate, cstate, coarse_new=cnew, theta=0.0)
    f1 = fstate.clone()
    fbat.step(fstate, fgrav, dtf, a0, am, f1)
    ffill.fill(f1, cstate, coarse_new=cnew, theta=0.5)
    f2 = f1.clone()
    fbat.step(f1, fgrav, dtf, am, a1, f2)
    csync = cnew.clone()
    sync.reflux(csync, reg)
    sync.average_down(csync, f2)
    torch.cuda.synchronize()
    counts = sync.counts()
    fbat.set_flux_register(None, 1, None)
    for x in (cfill, ffill, cbat, fbat):
        x.close()
    out = (_unpack(csync.cpu().numpy(), cdatas), _unpack(f2.cpu().numpy(), fdatas), counts)
    sync.close()
    return out


def _valid(a):
    return a[:, NG:-NG, NG:-NG, NG:-NG]


@pytest.mark.parametrize("groups", [False, True])
def test_fp64_sync_bitwise(nyx, reference, groups):
    prm = nyx.default_params()
    print("two-level sync fp64, groups", groups, flush=True)
    csync, fnew, counts = _gpu_two_levels(nyx, prm, reference["setup"], reference["dt_c"],
                                          groups)
    assert counts[0] == reference["nfaces"] and counts[2] == reference["ncov"]
    for a, b in zip(fnew, reference["fnew"]):
        assert np.array_equal(_valid(a), _valid(b))
    for a, b in zip(csync, reference["csync"]):
        assert np.array_equal(_valid(a), _valid(b))


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_sync_in_the_fused_launch_mode(nyx, reference, prec):
    # plans that feed flux registers keep the staged final stage but fuse the
    # x tracing and stage-0 solves: the same bits as the staged launches, and
    # (FP64) as the oracle
    p = nyx.NYX_FP64 if prec == "fp64" else nyx.NYX_MIXED
    prm = nyx.default_params(precision=p)
    print("two-level sync, fused mode,", prec, flush=True)
    runs = [_gpu_two_levels(nyx, prm, reference["setup"], reference["dt_c"], False, mode=m)
            for m in (nyx.NYX_LAUNCH_STAGED, nyx.NYX_LAUNCH_FUSED)]
    for a, b in zip(runs[0][0] + runs[0][1], runs[1][0] + runs[1][1]):
        assert np.array_equal(_valid(a), _valid(b))
    if prec == "fp64":
        for a, b in zip(runs[1][1], reference["fnew"]):
            assert np.array_equal(_valid(a), _valid(b))
        for a, b in zip(runs[1][0], reference["csync"]):
            assert np.array_equal(_valid(a), _valid(b))


def test_mixed_sync_close_and_conservative(nyx, reference):
    prm = nyx.default_params(precision=nyx.NYX_MIXED)
    print("two-level sync mixed", flush=True)
    csync, fnew, _ = _gpu_two_levels(nyx, prm, reference["setup"], reference["dt_c"], False)
    num = sum(np.abs(_valid(a) - _valid(b)).sum() for a, b in zip(csync, reference["csync"]))
    den = sum(np.abs(_valid(b)).sum() for b in reference["csync"])
    assert num / den <= 1e-5
    # the mixed path's own composite sums are conserved too: the register
    # holds the fluxes its updates used, up to their FP32 rounding
    cboxes, cdatas, fboxes, fdatas, cdom, _ = reference["setup"]
    before = composite_sums(cboxes, cdatas, fboxes, fdatas, cdom)
    after = composite_sums(cboxes, csync, fboxes, fnew, cdom)
    for c in range(5):
        assert abs(after[c][0] - before[c][0]) <= 1e-12 * before[c][1], c


def _random_layout(seed):
    """Coarse boxes: a grid of random cuts (multiples of 4) of a 16 x 24 x 16
    coarse domain; fine level: up to three non-overlapping boxes with even
    corners and extents (4 to 12 fine cells) anywhere in the 32 x 48 x 32
    fine domain, boundary included; fields as in two_level_setup."""
    rng = np.random.default_rng(seed)
    cdom, dom = (16, 24, 16), (32, 48, 32)
    cuts = []
    for n in cdom:
        c, x = [0], 0
        while x < n:
            x = min(n, x + 4 * int(rng.integers(1, 3)))
            c.append(x)
        cuts.append(c)
    cboxes = []
    for z0, z1 in zip(cuts[2][:-1], cuts[2][1:]):
        for y0, y1 in zip(cuts[1][:-1], cuts[1][1:]):
            for x0, x1 in zip(cuts[0][:-1], cuts[0][1:]):
                cboxes.append(((x1 - x0, y1 - y0, z1 - z0), (x0, y0, z0)))
    used = np.zeros(cdom[::-1], dtype=bool)
    fboxes = []
    for _ in range(40):
        if len(fboxes) == 3:
            break
        n = tuple(2 * int(rng.integers(2, 7)) for _ in range(3))
        lo = tuple(2 * int(rng.integers(0, (dom[d] - n[d]) // 2 + 1)) for d in range(3))
        sl = tuple(slice(lo[d] // 2, (lo[d] + n[d]) // 2) for d in (2, 1, 0))
        if used[sl].any():
            continue
        used[sl] = True
        fboxes.append((n, lo))
    return _fields(rng, cboxes, fboxes, cdom, dom)


def _fields(rng, cboxes, fboxes, cdom, dom):
    """Fields of the layout as in two_level_setup: a random coarse state, the
    fine level injected from it with a perturbed density."""
    shape = cdom[::-1]
    rho = synth.lognormal(rng, shape, 1.0, 0.5)
    u = rng.normal(0.0, 0.3, (3,) + shape)
    p = synth.lognormal(rng, shape, 0.6, 0.3)
    Uc = synth.conserved(rho, u, p, 0.5)
    cdatas = []
    for n, lo in cboxes:
        a = np.zeros((6,) + tuple(x + 2 * NG for x in n[::-1]))
        _valid(a)[...] = Uc[:, lo[2]:lo[2] + n[2], lo[1]:lo[1] + n[1], lo[0]:lo[0] + n[0]]
        cdatas.append(a)
    fdatas = []
    for n, lo in fboxes:
        a = np.zeros((6,) + tuple(x + 2 * NG for x in n[::-1]))
        cl = [x // 2 for x in lo]
        blk = Uc[:, cl[2]:cl[2] + n[2] // 2, cl[1]:cl[1] + n[1] // 2, cl[0]:cl[0] + n[0] // 2]
        v = blk.repeat(2, axis=1).repeat(2, axis=2).repeat(2, axis=3)
        v[0] = v[0] * (1.0 + 0.1 * rng.uniform(-1, 1, v.shape[1:]))
        _valid(a)[...] = v
        fdatas.append(a)
    return cboxes, cdatas, fboxes, fdatas, cdom, dom


@pytest.mark.parametrize("seed", [31, 32, 33])
def test_fp64_sync_random_layouts_bitwise(nyx, seed):
    setup = _random_layout(seed)
    cboxes, cdatas, fboxes, fdatas, cdom, dom = setup
    print("random two-level layout", seed, len(cboxes), "coarse,", len(fboxes), "fine", flush=True)
    cnew, fnew, cflux, ffl, dt_c, dt_f, _ = advance_two_levels(cboxes, cdatas, fboxes, fdatas,
                                                               cdom, dom)
    csync = [x.copy() for x in cnew]
    nf, nc = oracle.reflux_average_down(cboxes, NG, 1.0 / cdom[0], csync, cflux, dt_c, fboxes,
                                        NG, dom, fnew, ffl, dt_f)
    got_c, got_f, counts = _gpu_two_levels(nyx, nyx.default_params(), setup, dt_c, False)
    assert counts[0] == nf and counts[2] == nc
    for a, b in zip(got_f, fnew):
        assert np.array_equal(_valid(a), _valid(b))
    for a, b in zip(got_c, csync):
        assert np.array_equal(_valid(a), _valid(b))



def test_fp64_fine_level_covering_the_domain(nyx):
    """The degenerate layout with no coarse-fine interface: the fine level
    covers the whole domain, so the plan has no register faces and no reflux
    cells, every fine ghost is a copy, and the synchronisation is the
    average-down alone; still equal to the oracle bit for bit."""
    rng = np.random.default_rng(35)
    cdom, dom = (8, 12, 8), (16, 24, 16)
    cboxes = [((8, 12, 4), (0, 0, 0)), ((8, 12, 4), (0, 0, 4))]
    fboxes = [((16, 24, 6), (0, 0, 0)), ((16, 24, 4), (0, 0, 6)), ((16, 24, 6), (0, 0, 10))]
    setup = _fields(rng, cboxes, fboxes, cdom, dom)
    cboxes, cdatas, fboxes, fdatas, cdom, dom = setup
    print("fine level covering the domain", flush=True)
    cnew, fnew, cflux, ffl, dt_c, dt_f, _ = advance_two_levels(cboxes, cdatas, fboxes, fdatas,
                                                               cdom, dom)
    csync = [x.copy() for x in cnew]
    nf, nc = oracle.reflux_average_down(cboxes, NG, 1.0 / cdom[0], csync, cflux, dt_c, fboxes,
                                        NG, dom, fnew, ffl, dt_f)
    assert nf == 0 and nc == 8 * 12 * 8
    got_c, got_f, counts = _gpu_two_levels(nyx, nyx.default_params(), setup, dt_c, False)
    assert counts == (0, 0, nc)
    for a, b in zip(got_f, fnew):
        assert np.array_equal(_valid(a), _valid(b))
    for a, b in zip(got_c, csync):
        assert np.array_equal(_valid(a), _valid(b))

def test_two_level_cycle_graph_replay_matches_eager(nyx, reference):
    """Two two-level cycles (coarse fills and step feeding the register, fine
    fills in time and two substeps, reflux, average-down; the coarse state
    ping-pongs between two buffers) captured in one HIP graph: every replay,
    with unrelated eager work between replays, equals the eager sequence bit
    for bit."""
    import torch
    prm = nyx.default_params()
    cboxes, cdatas, fboxes, fdatas, cdom, dom = reference["setup"]
    dt_c = reference["dt_c"]
    clo = [lo for _, lo in cboxes]
    flo = [lo for _, lo in fboxes]
    cb, cflat, cg = _pack(nyx, cboxes, cdatas, 1.0 / cdom[0])
    fb, fflat, fg = _pack(nyx, fboxes, fdatas, 1.0 / dom[0])
    cgrav = torch.zeros(cg, dtype=torch.float64, device="cuda")
    fgrav = torch.zeros(fg, dtype=torch.float64, device="cuda")
    cfill = nyx.FillPlan(cb, clo, cdom)
    ffill = nyx.FillPlan(fb, flo, dom, coarse=(cb, clo))
    sync = nyx.SyncPlan((fb, flo), (cb, clo), dom)
    reg = sync.register()
    cbat = nyx.Batch(prm, cb, aligned_ws(nyx.Batch.workspace_bytes(prm, cb)[1]))
    fbat = nyx.Batch(prm, fb, aligned_ws(nyx.Batch.workspace_bytes(prm, fb)[1]))
    cbat.set_flux_register(sync, 0, reg)
    fbat.set_flux_register(sync, 1, reg)
    dtc = torch.full((len(cb),), dt_c, dtype=torch.float64, device="cuda")
    dtf = torch.full((len(fb),), 0.5 * dt_c, dtype=torch.float64, device="cuda")
    a = [0.5 + 0.0025 * k for k in range(5)]

    def cycle(c, c2, f, f2, k):
        reg.zero_()
        cfill.fill(c)
        cbat.step(c, cgrav, dtc, a[2 * k], a[2 * k + 2], c2)
        cfill.fill(c2)
        ffill.fill(f, c, coarse_new=c2, theta=0.0)
        fbat.step(f, fgrav, dtf, a[2 * k], a[2 * k + 1], f2)
        ffill.fill(f2, c, coarse_new=c2, theta=0.5)
        fbat.step(f2, fgrav, dtf, a[2 * k + 1], a[2 * k + 2], f)
        sync.reflux(c2, reg)
        sync.average_down(c2, f)

    def two_cycles(bufs):
        c, c2, f, f2 = bufs
        cycle(c, c2, f, f2, 0)
        cycle(c2, c, f, f2, 1)

    def fresh():
        return [to_dev(cflat), to_dev(cflat), to_dev(fflat), to_dev(fflat)]

    eager, E = [], fresh()
    for r in range(3):
        two_cycles(E)
        torch.cuda.synchronize()
        eager.append((E[0].cpu().numpy().copy(), E[2].cpu().numpy().copy()))
    Gb = fresh()
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            two_cycles(Gb)
    torch.cuda.synchronize()
    for r in range(3):
        g.replay()
        torch.cuda.synchronize()
        _ = (Gb[1] * 1.0).sum().item()  # unrelated eager work between replays
        assert np.array_equal(Gb[0].cpu().numpy(), eager[r][0]), r
        assert np.array_equal(Gb[2].cpu().numpy(), eager[r][1]), r
    fbat.set_flux_register(None, 1, None)
    cbat.set_flux_register(None, 0, None)
    for x in (cfill, ffill, cbat, fbat, sync):
        x.close()


def test_fp64_sync_fine_slab_spanning_the_periodic_axis(nyx):
    # a fine box that spans the whole domain along x: no interface faces
    # across x (its x neighbours are its own periodic images)
    setup = list(_random_layout(41))
    cboxes, cdatas, _, _, cdom, dom = setup
    rng = np.random.default_rng(41)
    fboxes = [((32, 8, 6), (0, 10, 12))]
    shape = cdom[::-1]
    Uc = synth.conserved(synth.lognormal(rng, shape, 1.0, 0.5), rng.normal(0, 0.3, (3,) + shape),
                         synth.lognormal(rng, shape, 0.6, 0.3), 0.5)
    for (n, lo), a in zip(cboxes, cdatas):
        _valid(a)[...] = Uc[:, lo[2]:lo[2] + n[2], lo[1]:lo[1] + n[1], lo[0]:lo[0] + n[0]]
    n, lo = fboxes[0]
    a = np.zeros((6,) + tuple(x + 2 * NG for x in n[::-1]))
    cl = [x // 2 for x in lo]
    blk = Uc[:, cl[2]:cl[2] + n[2] // 2, cl[1]:cl[1] + n[1] // 2, cl[0]:cl[0] + n[0] // 2]
    _valid(a)[...] = blk.repeat(2, axis=1).repeat(2, axis=2).repeat(2, axis=3)
    setup = (cboxes, cdatas, fboxes, [a], cdom, dom)
    cnew, fnew, cflux, ffl, dt_c, dt_f, _ = advance_two_levels(*setup)
    csync = [x.copy() for x in cnew]
    nf, nc = oracle.reflux_average_down(cboxes, NG, 1.0 / cdom[0], csync, cflux, dt_c, fboxes,
                                        NG, dom, fnew, ffl, dt_f)
    assert nf == 2 * (16 * 3) + 2 * (16 * 4)  # y and z faces of the 16 x 4 x 3 coarse slab
    got_c, got_f, counts = _gpu_two_levels(nyx, nyx.default_params(), setup, dt_c, False)
    assert counts[0] == nf and counts[2] == nc
    for x, y in zip(got_f, fnew):
        assert np.array_equal(_valid(x), _valid(y))
    for x, y in zip(got_c, csync):
        assert np.array_equal(_valid(x), _valid(y))
