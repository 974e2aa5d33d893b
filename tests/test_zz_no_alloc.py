"""The allocation-free single-box step (nyx_hydro_step_noalloc) against the
workspace entry point (nyx_hydro_step) through the C ABI: the same kernels on
the same inputs, so the new state, the next dt and the counters must be equal
bit for bit.  Two calls in a row, the second on a smaller box, show that the
shared scratch array carries nothing from one call into the next."""
import numpy as np
import pytest

from gpu_harness import NG, aligned_ws, to_dev
from paper_1301_4498_amd import synth

pytestmark = pytest.mark.gpu


def _both(nyx, torch, prm, n, seed, a0=0.5, a1=0.5025):
    U0, g = synth.random_box(n, seed=seed, a=a0, kind=1)
    dx = 1.0 / n[0]
    box = nyx.make_box(n, NG, dx)
    gdt = torch.float64 if prm.precision == nyx.NYX_FP64 else torch.float32
    Ui = to_dev(U0)
    G = to_dev(g, gdt)
    out = []
    for noalloc in (True, False):
        Uo = torch.zeros_like(Ui)
        dtn = torch.zeros(1, dtype=torch.float64, device="cuda")
        st = torch.zeros(10, dtype=torch.int64, device="cuda")
        dt = 0.2 * dx * a0
        print("noalloc=%s n=%s seed=%d precision=%d" % (noalloc, n, seed, prm.precision),
              flush=True)
        if noalloc:
            nyx.hydro_step_noalloc(prm, box, Ui, G, dt, a0, a1, Uo, dt_next=dtn, stats=st)
        else:
            ws = aligned_ws(nyx.workspace_bytes(prm, box))
            nyx.hydro_step(prm, box, Ui, G, dt, a0, a1, Uo, dt_next=dtn, stats=st, workspace=ws)
        torch.cuda.synchronize()
        v = Uo.cpu().numpy()[:, NG:-NG, NG:-NG, NG:-NG]
        out.append((v, float(dtn.item()), nyx.stats_dict(st)))
    return out


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_step_equals_workspace_step(precision):
    import torch

    import paper_1301_4498_amd as nyx
    prm = nyx.default_params(precision=nyx.NYX_FP64 if precision == "fp64" else nyx.NYX_MIXED)
    # a 32^3 box, then a smaller ragged one
    for n, seed in (((32, 32, 32), 11), ((14, 10, 18), 12)):
        (a, dta, sa), (b, dtb, sb) = _both(nyx, torch, prm, n, seed)
        assert np.array_equal(a, b), (n, np.abs(a - b).max())
        assert dta == dtb and dta > 0.0
        assert sa == sb
        assert sa["riemann_calls"] > 0 and sa["nonfinite"] == 0
