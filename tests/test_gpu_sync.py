"""Two-level synchronisation through the C ABI (Sec. 4.3: flux registers fed
by the batched steps, nyx_reflux, nyx_average_down) against the oracle.  One
coarse step of eight 8^3 boxes and two fine substeps of three fine boxes
(with a fine-fine face and neighbours across the periodic boundary), fine
ghosts filled from the coarse level at the old and at the mid time.  FP64:
the synchronised coarse level and the fine level equal the oracle's bit for
bit, with the plan split into one or several workspace groups; FP32-mixed:
within 1e-5 relative L1, and its composite sums conserved."""
import numpy as np
import pytest

import oracle
from gpu_harness import NG, aligned_ws, to_dev
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


def _gpu_two_levels(nyx, prm, setup, dt_c, groups, a0=0.5, a1=0.505):
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
    cbat.set_flux_register(sync, 0, reg)
    fbat.set_flux_register(sync, 1, reg)
    dtc = torch.full((len(cb),), dt_c, dtype=torch.float64, device="cuda")
    dtf = torch.full((len(fb),), 0.5 * dt_c, dtype=torch.float64, device="cuda")
    am = 0.5 * (a0 + a1)
    cfill.fill(cstate)
    cnew = cstate.clone()
    cbat.step(cstate, cgrav, dtc, a0, a1, cnew)
    cfill.fill(cnew)
    cmid = 0.5 * (cstate + cnew)
    ffill.fill(fstate, cstate)
    f1 = fstate.clone()
    fbat.step(fstate, fgrav, dtf, a0, am, f1)
    ffill.fill(f1, cmid)
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
