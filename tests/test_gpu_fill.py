"""Ghost fill of an AMR level through the C ABI (nyx_fill_plan_*,
nyx_fill_level) against the oracle's fill: same-level copies between uneven
boxes and their periodic images, coarse-fine limited linear interpolation
from a coarse level of several boxes, boxes at the domain boundary, random
layouts; bitwise equal arrays and equal copied / interpolated counts.  At
full size, 512 patches of 64^3 tiling a 512^3 domain reproduce the
periodic padding of the domain exactly."""
import numpy as np
import pytest

import oracle
from gpu_harness import NG, to_dev
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


def _split(dom, cuts):
    edges = [[0] + list(c) + [d] for c, d in zip(cuts, dom)]
    out = []
    for z0, z1 in zip(edges[2][:-1], edges[2][1:]):
        for y0, y1 in zip(edges[1][:-1], edges[1][1:]):
            for x0, x1 in zip(edges[0][:-1], edges[0][1:]):
                out.append(((x1 - x0, y1 - y0, z1 - z0), (x0, y0, z0)))
    return out


def _pack(nyx, layout, arrays, dx=1.0):
    boxes, off = [], 0
    for (n, lo), a in zip(layout, arrays):
        boxes.append(nyx.make_box(n, NG, dx, state_off=off))
        off += a.size
    return boxes, np.concatenate([a.ravel() for a in arrays])


def _unpack(flat, arrays):
    out, off = [], 0
    for a in arrays:
        out.append(flat[off:off + a.size].reshape(a.shape))
        off += a.size
    return out


def _gpu_fill(nyx, layout, arrays, dom, coarse=None, coarse_new=None, theta=0.0):
    """coarse: None or (clayout, carrays) with filled ghosts; coarse_new: the
    coarse arrays at the end of the step (time interpolation by theta)."""
    boxes, flat = _pack(nyx, layout, arrays)
    cplan_arg, cflat, cnew = None, None, None
    if coarse is not None:
        clayout, carrays = coarse
        cboxes, cf = _pack(nyx, clayout, carrays, 2.0)
        cplan_arg = (cboxes, [lo for _, lo in clayout])
        cflat = to_dev(cf)
        if coarse_new is not None:
            cnew = to_dev(_pack(nyx, clayout, coarse_new, 2.0)[1])
    plan = nyx.FillPlan(boxes, [lo for _, lo in layout], dom, coarse=cplan_arg)
    T = to_dev(flat)
    plan.fill(T, cflat, ncomp=arrays[0].shape[0], coarse_new=cnew, theta=theta)
    import torch
    torch.cuda.synchronize()
    counts = plan.counts()
    plan.close()
    return _unpack(T.cpu().numpy(), arrays), counts


def _with_blank_ghosts(layout, ncomp, rng):
    arrs = []
    for n, _ in layout:
        a = np.full((ncomp, n[2] + 8, n[1] + 8, n[0] + 8), -7.0)
        a[:, NG:-NG, NG:-NG, NG:-NG] = rng.normal(size=(ncomp, n[2], n[1], n[0]))
        arrs.append(a)
    return arrs


def test_same_level_uneven_tiling(nyx):
    rng = np.random.default_rng(11)
    dom = (24, 16, 20)
    field = rng.normal(size=(6, dom[2], dom[1], dom[0]))
    pad = synth.pad_periodic(field, NG)
    layout = _split(dom, [(10, 16), (6,), (8, 12)])
    arrays = []
    for n, lo in layout:
        a = np.full((6, n[2] + 8, n[1] + 8, n[0] + 8), -7.0)
        a[:, NG:-NG, NG:-NG, NG:-NG] = field[:, lo[2]:lo[2] + n[2], lo[1]:lo[1] + n[1],
                                             lo[0]:lo[0] + n[0]]
        arrays.append(a)
    got, (nc, ni) = _gpu_fill(nyx, layout, arrays, dom)
    ref = [a.copy() for a in arrays]
    rc, ri = oracle.fill_level(layout, NG, dom, ref)
    assert (nc, ni) == (rc, ri) and ni == 0
    for (n, lo), g, r in zip(layout, got, ref):
        assert np.array_equal(g, r)
        want = pad[:, lo[2]:lo[2] + n[2] + 8, lo[1]:lo[1] + n[1] + 8, lo[0]:lo[0] + n[0] + 8]
        assert np.array_equal(g, want)


@pytest.mark.parametrize("case", ["pair_in_one_coarse_box", "boundary_and_eight_coarse_boxes",
                                  "random_layout"])
def test_two_level_fill_matches_oracle(nyx, case):
    rng = np.random.default_rng({"pair_in_one_coarse_box": 1, "boundary_and_eight_coarse_boxes": 2,
                                 "random_layout": 3}[case])
    if case == "pair_in_one_coarse_box":
        dom, clayout = (24, 24, 24), [((12, 12, 12), (0, 0, 0))]
        layout = [((8, 8, 8), (4, 8, 8)), ((8, 8, 8), (12, 8, 8))]
    elif case == "boundary_and_eight_coarse_boxes":
        dom = (32, 32, 32)
        clayout = _split((16, 16, 16), [(8,), (8,), (8,)])
        layout = [((8, 8, 8), (24, 0, 12)), ((6, 6, 6), (2, 2, 2))]
    else:
        dom = (64, 64, 64)
        clayout = _split((32, 32, 32), [(8, 16, 24)] * 3)
        layout = []
        while len(layout) < 10:
            n = tuple(int(2 * rng.integers(1, 7)) for _ in range(3))
            lo = tuple(int(2 * rng.integers(0, 26)) for _ in range(3))
            if any(lo[d] + n[d] > 64 for d in range(3)):
                continue
            if any(all(lo[d] < l2[d] + n2[d] and l2[d] < lo[d] + n[d] for d in range(3))
                   for n2, l2 in layout):
                continue
            layout.append((n, lo))
    cdom = tuple(d // 2 for d in dom)
    # coarse level: random fields, ghosts filled by the oracle's own level fill
    cfield = np.exp(rng.normal(0, 0.5, size=(6,) + cdom[::-1]))
    cpad = synth.pad_periodic(cfield, NG)
    carrays = [cpad[:, lo[2]:lo[2] + n[2] + 8, lo[1]:lo[1] + n[1] + 8, lo[0]:lo[0] + n[0] + 8].copy()
               for n, lo in clayout]
    arrays = _with_blank_ghosts(layout, 6, rng)
    got, (nc, ni) = _gpu_fill(nyx, layout, arrays, dom, coarse=(clayout, carrays))
    ref = [a.copy() for a in arrays]
    rc, ri = oracle.fill_level(layout, NG, dom, ref, coarse=(clayout, NG, carrays))
    assert (nc, ni) == (rc, ri) and ni > 0, (nc, ni, rc, ri)
    for g, r in zip(got, ref):
        assert np.array_equal(g, r)


def test_full_size_patch_grid_reproduces_periodic_padding(nyx):
    # 512 patches of 64^3 tiling the 512^3 stress domain (the benchmark's
    # patch layout): every ghost cell is a copy
    import torch
    state, _ = synth.stress_fields_torch(n=512)
    g8, m = (8, 8, 8), 64
    parts = synth.split_patches(state, g8)
    want = torch.cat([p.reshape(-1) for p in parts])
    T = want.clone()
    P = (m + 8) ** 3
    Tv = T.view(512, 6, m + 8, m + 8, m + 8)
    Tv[:, :, :NG] = -1.0
    Tv[:, :, -NG:] = -1.0
    Tv[:, :, :, :NG] = -1.0
    Tv[:, :, :, -NG:] = -1.0
    Tv[:, :, :, :, :NG] = -1.0
    Tv[:, :, :, :, -NG:] = -1.0
    boxes = [nyx.make_box((m, m, m), NG, 1.0 / 512, state_off=6 * P * b) for b in range(512)]
    lo = [(m * (b % 8), m * ((b // 8) % 8), m * (b // 64)) for b in range(512)]
    plan = nyx.FillPlan(boxes, lo, (512, 512, 512))
    nc, ni = plan.counts()
    assert ni == 0 and nc == 512 * ((m + 8) ** 3 - m ** 3)
    plan.fill(T)
    torch.cuda.synchronize()
    assert torch.equal(T, want)
    plan.close()


@pytest.mark.parametrize("theta", [0.0, 0.25, 0.5, 1.0])
def test_two_level_fill_in_time_matches_oracle(nyx, theta):
    # subcycling: the coarse data at fraction theta of the coarse step
    rng = np.random.default_rng(21)
    dom = (32, 32, 32)
    clayout = _split((16, 16, 16), [(8,), (8,), (8,)])
    layout = [((8, 8, 8), (24, 0, 12)), ((6, 6, 6), (2, 2, 2)), ((10, 4, 6), (10, 20, 20))]
    c0 = synth.pad_periodic(np.exp(rng.normal(0, 0.5, size=(6, 16, 16, 16))), NG)
    c1 = synth.pad_periodic(np.exp(rng.normal(0, 0.5, size=(6, 16, 16, 16))), NG)
    cut = lambda cp: [cp[:, lo[2]:lo[2] + n[2] + 8, lo[1]:lo[1] + n[1] + 8,
                         lo[0]:lo[0] + n[0] + 8].copy() for n, lo in clayout]
    arrays = _with_blank_ghosts(layout, 6, rng)
    got, (nc, ni) = _gpu_fill(nyx, layout, arrays, dom, coarse=(clayout, cut(c0)),
                              coarse_new=cut(c1), theta=theta)
    ref = [a.copy() for a in arrays]
    rc, ri = oracle.fill_level(layout, NG, dom, ref, coarse=(clayout, NG, cut(c0)),
                               coarse_new=cut(c1), theta=theta)
    assert (nc, ni) == (rc, ri) and ni > 0
    for g, r in zip(got, ref):
        assert np.array_equal(g, r)
