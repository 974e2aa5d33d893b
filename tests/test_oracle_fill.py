"""Pins of the oracle's level ghost fill (Sec. 4.1: ghost cells, and the
conservative limited piecewise-linear interpolation from the coarser level),
no GPU: same-level copies reproduce the periodic padding of the domain; the
interpolation is exact for linear data, conserves every coarse cell's
average over its eight children and creates no new extrema; a ghost cell
covered by neither level is an error."""
import numpy as np
import pytest

import oracle
from paper_1301_4498_amd import synth

NG = 4


def _split(dom_cells, cuts):
    """Boxes (n, lo) tiling [0, dom) with the given cut positions per axis."""
    edges = [[0] + list(c) + [d] for c, d in zip(cuts, dom_cells)]
    out = []
    for z0, z1 in zip(edges[2][:-1], edges[2][1:]):
        for y0, y1 in zip(edges[1][:-1], edges[1][1:]):
            for x0, x1 in zip(edges[0][:-1], edges[0][1:]):
                out.append(((x1 - x0, y1 - y0, z1 - z0), (x0, y0, z0)))
    return out


def _cut(padded_dom, n, lo, ng=NG):
    """The padded box (n, lo) cut from a periodically padded domain array."""
    return padded_dom[:, lo[2]:lo[2] + n[2] + 2 * ng, lo[1]:lo[1] + n[1] + 2 * ng,
                      lo[0]:lo[0] + n[0] + 2 * ng].copy()


def _blank_ghosts(a, ng=NG):
    b = np.full_like(a, np.nan)
    b[:, ng:-ng, ng:-ng, ng:-ng] = a[:, ng:-ng, ng:-ng, ng:-ng]
    return b


def test_same_level_copies_reproduce_periodic_padding():
    rng = np.random.default_rng(1)
    dom = (24, 16, 20)
    field = rng.normal(size=(6, dom[2], dom[1], dom[0]))
    pad = synth.pad_periodic(field, NG)
    boxes = _split(dom, [(10, 16), (6,), (8, 12)])  # uneven, some narrower than the ghost width
    datas = [_blank_ghosts(_cut(pad, n, lo)) for n, lo in boxes]
    ncp, nip = oracle.fill_level(boxes, NG, dom, datas)
    assert nip == 0 and ncp == sum((n[0] + 8) * (n[1] + 8) * (n[2] + 8) - n[0] * n[1] * n[2]
                                   for n, _ in boxes)
    for (n, lo), d in zip(boxes, datas):
        assert np.array_equal(d, _cut(pad, n, lo)), (n, lo)


def test_single_box_is_its_own_periodic_image():
    rng = np.random.default_rng(2)
    dom = (6, 8, 4)  # the box is narrower than two ghost widths
    field = rng.normal(size=(6, dom[2], dom[1], dom[0]))
    pad = synth.pad_periodic(field, NG)
    d = _blank_ghosts(pad.copy())
    oracle.fill_level([(dom, (0, 0, 0))], NG, dom, [d])
    assert np.array_equal(d, pad)


def _two_levels(cfield, fine_boxes, cdom):
    """Coarse level = one box over the coarse domain with periodic ghosts;
    fine boxes start with blank ghosts."""
    cpad = synth.pad_periodic(cfield, NG)
    fdata = []
    for n, lo in fine_boxes:
        a = np.full((cfield.shape[0], n[2] + 8, n[1] + 8, n[0] + 8), np.nan)
        a[:, NG:-NG, NG:-NG, NG:-NG] = 0.0
        fdata.append(a)
    return ([(cdom, (0, 0, 0))], NG, [cpad]), fdata


def test_interpolation_exact_for_linear_data():
    # coarse data linear in the cell index: unlimited slopes, alpha = 1, and
    # the fine values are the linear function at the fine cell centres; the
    # coarse box's ghost cells continue the linear function (not periodic)
    cdom = (16, 16, 16)
    a, b = 0.7, np.array([0.11, -0.05, 0.031])
    K, J, I = np.meshgrid(*[np.arange(-NG, 16 + NG)] * 3, indexing="ij")
    clin = a + b[0] * I + b[1] * J + b[2] * K
    cpad = np.stack([clin, 2.0 * clin])
    fine = [((8, 8, 8), (12, 10, 14))]  # interior: its ghost cells are all coarse-covered
    fdata = [np.zeros((2, 16, 16, 16))]
    ncp, nip = oracle.fill_level(fine, NG, (32, 32, 32), fdata, coarse=([(cdom, (0, 0, 0))], NG, [cpad]),
                                 ncomp=2)
    assert ncp == 0 and nip == 16 ** 3 - 8 ** 3
    (n, lo), d = fine[0], fdata[0]
    k, j, i = np.meshgrid(*[np.arange(-NG, 8 + NG)] * 3, indexing="ij")
    # fine cell centre in coarse index units: (g + 1/2) / 2 - 1/2
    X = (lo[0] + i + 0.5) / 2 - 0.5
    Y = (lo[1] + j + 0.5) / 2 - 0.5
    Z = (lo[2] + k + 0.5) / 2 - 0.5
    want = a + b[0] * X + b[1] * Y + b[2] * Z
    ghost = np.ones((16, 16, 16), bool)
    ghost[NG:-NG, NG:-NG, NG:-NG] = False
    assert np.allclose(d[0][ghost], want[ghost], rtol=0, atol=1e-13)
    assert np.allclose(d[1][ghost], 2.0 * want[ghost], rtol=0, atol=1e-13)


def test_interpolation_conserves_and_creates_no_extrema():
    rng = np.random.default_rng(3)
    cdom = (12, 12, 12)
    cfield = np.exp(rng.normal(0, 1.0, size=(1,) + cdom))
    coarse, fdata = _two_levels(cfield, [((8, 8, 8), (8, 8, 8))], cdom)
    cpad = coarse[2][0]
    oracle.fill_level([((8, 8, 8), (8, 8, 8))], NG, (24, 24, 24), fdata, coarse=coarse, ncomp=1)
    d = fdata[0][0]
    lo = np.array([8, 8, 8])
    # every coarse cell whose eight children all lie in the ghost layer:
    # global coarse index X with children 2X..2X+1 inside [lo-4, lo+12)
    checked = 0
    for Z in range(2, 10):
        for Y in range(2, 10):
            for X in range(2, 10):
                kids = []
                for dz in (0, 1):
                    for dy in (0, 1):
                        for dx in (0, 1):
                            g = np.array([2 * X + dx, 2 * Y + dy, 2 * Z + dz])
                            loc = g - lo + NG
                            inside = np.all((g >= lo) & (g < lo + 8))
                            if inside:
                                break
                            kids.append(d[loc[2], loc[1], loc[0]])
                if len(kids) < 8:
                    continue
                u0 = cpad[0, Z + NG, Y + NG, X + NG]
                nb = [cpad[0, Z + NG + dz, Y + NG + dy, X + NG + dx]
                      for dz, dy, dx in ((0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0),
                                         (0, 0, 1), (0, 0, -1))]
                assert np.mean(kids) == pytest.approx(u0, rel=1e-14)
                assert min(kids) >= min(nb) * (1 - 1e-14) and max(kids) <= max(nb) * (1 + 1e-14)
                checked += 1
    assert checked > 100


def test_copies_take_precedence_and_improper_nesting_is_an_error():
    rng = np.random.default_rng(4)
    cdom = (12, 12, 12)
    cfield = rng.normal(size=(1,) + cdom)
    boxes = [((8, 8, 8), (4, 8, 8)), ((8, 8, 8), (12, 8, 8))]  # two fine boxes side by side
    coarse, fdata = _two_levels(cfield, boxes, cdom)
    rng2 = np.random.default_rng(5)
    for a in fdata:
        a[:, NG:-NG, NG:-NG, NG:-NG] = rng2.normal(size=(1, 8, 8, 8))
    ncp, nip = oracle.fill_level(boxes, NG, (24, 24, 24), fdata, coarse=coarse, ncomp=1)
    face = 4 * 8 * 8  # each box sees the other's 4 x 8 x 8 face cells
    assert ncp == 2 * face
    assert nip == 2 * (16 ** 3 - 8 ** 3) - ncp
    # the shared face holds the neighbour's valid cells
    assert np.array_equal(fdata[0][:, NG:-NG, NG:-NG, -NG:], fdata[1][:, NG:-NG, NG:-NG, NG:2 * NG])
    # with no coarse level the open faces are covered by nothing
    with pytest.raises(ValueError):
        oracle.fill_level(boxes, NG, (24, 24, 24), [a.copy() for a in fdata], ncomp=1)


def test_time_interpolation_of_the_coarse_data():
    # subcycling (Sec. 4.2): with coarse data linear in space at the start and
    # at the end of the coarse step, the ghost cells at fraction theta of the
    # step are the linear field interpolated in time
    cdom = (16, 16, 16)
    K, J, I = np.meshgrid(*[np.arange(-NG, 16 + NG)] * 3, indexing="ij")
    c0 = (0.7 + 0.11 * I - 0.05 * J + 0.031 * K)[None]
    c1 = (1.3 - 0.02 * I + 0.09 * J + 0.017 * K)[None]
    fine = [((8, 8, 8), (12, 10, 14))]
    k, j, i = np.meshgrid(*[np.arange(-NG, 8 + NG)] * 3, indexing="ij")
    lo = fine[0][1]
    X = (lo[0] + i + 0.5) / 2 - 0.5
    Y = (lo[1] + j + 0.5) / 2 - 0.5
    Z = (lo[2] + k + 0.5) / 2 - 0.5
    ghost = np.ones((16, 16, 16), bool)
    ghost[NG:-NG, NG:-NG, NG:-NG] = False
    for theta in (0.0, 0.25, 0.5, 1.0):
        d = [np.zeros((1, 16, 16, 16))]
        oracle.fill_level(fine, NG, (32, 32, 32), d, coarse=([(cdom, (0, 0, 0))], NG, [c0]),
                          ncomp=1, coarse_new=[c1], theta=theta)
        w0 = 0.7 + 0.11 * X - 0.05 * Y + 0.031 * Z
        w1 = 1.3 - 0.02 * X + 0.09 * Y + 0.017 * Z
        want = (1 - theta) * w0 + theta * w1
        assert np.allclose(d[0][0][ghost], want[ghost], rtol=0, atol=1e-13), theta
    # theta = 0 is the fill from the old data, bit for bit
    a, b = [np.zeros((1, 16, 16, 16))], [np.zeros((1, 16, 16, 16))]
    rng = np.random.default_rng(8)
    r0 = np.exp(rng.normal(0, 1, (1,) + cdom))
    r1 = np.exp(rng.normal(0, 1, (1,) + cdom))
    p0, p1 = synth.pad_periodic(r0, NG), synth.pad_periodic(r1, NG)
    oracle.fill_level(fine, NG, (32, 32, 32), a, coarse=([(cdom, (0, 0, 0))], NG, [p0]), ncomp=1)
    oracle.fill_level(fine, NG, (32, 32, 32), b, coarse=([(cdom, (0, 0, 0))], NG, [p0]), ncomp=1,
                      coarse_new=[p1], theta=0.0)
    assert np.array_equal(a[0], b[0])
    # the children of a coarse cell average to its time-interpolated value
    c = [np.zeros((1, 16, 16, 16))]
    oracle.fill_level(fine, NG, (32, 32, 32), c, coarse=([(cdom, (0, 0, 0))], NG, [p0]), ncomp=1,
                      coarse_new=[p1], theta=0.3)
    # coarse cell (5, 4, 6): children x 10..11, y 8..9, z 12..13 are ghosts of the fine box
    kids = c[0][0, 12 - lo[2] + NG:14 - lo[2] + NG, 8 - lo[1] + NG:10 - lo[1] + NG,
                10 - lo[0] + NG:12 - lo[0] + NG]
    u = p0[0, 6 + NG, 4 + NG, 5 + NG] + 0.3 * (p1[0, 6 + NG, 4 + NG, 5 + NG] - p0[0, 6 + NG, 4 + NG, 5 + NG])
    assert kids.shape == (2, 2, 2) and kids.mean() == pytest.approx(u, rel=1e-14)
    with pytest.raises(ValueError):
        oracle.fill_level(fine, NG, (32, 32, 32), c, coarse=([(cdom, (0, 0, 0))], NG, [p0]),
                          ncomp=1, coarse_new=[p1], theta=1.5)
