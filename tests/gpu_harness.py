"""Helpers of the GPU tests: drive the HIP library through its binding and the
oracle through its own wrapper on the same seeded inputs.  The two sides share
only the inputs."""
from __future__ import annotations

import numpy as np

import oracle
from paper_1301_4498_amd import synth

NG = 4


def torch_mod():
    import torch
    return torch


def aligned_ws(nbytes: int):
    """A uint8 device buffer of nbytes whose address is 256-byte aligned."""
    torch = torch_mod()
    t = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    off = (-t.data_ptr()) % 256
    return t[off:off + nbytes]


def to_dev(a: np.ndarray, dtype=None):
    torch = torch_mod()
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda")


def oracle_run(state, grav, dx, a_list, params=None, dts=None, cfl=0.5, periodic=True):
    """Advance len(a_list)-1 steps on the oracle; returns (state, dts, stats list).
    dts: if None, each step's dt is the oracle's CFL step."""
    params = params or oracle.Params()
    U = state.copy()
    out_dts, stats = [], []
    for k in range(len(a_list) - 1):
        dt = oracle.estimate_dt(U, NG, a_list[k], dx, cfl, params) if dts is None else dts[k]
        U, st = oracle.hydro_step(U, grav, NG, dt, dx, a_list[k], a_list[k + 1], params)
        if periodic:
            synth.fill_periodic_inplace(U)
        out_dts.append(dt)
        stats.append(st)
    return U, out_dts, stats


def gpu_run(state, grav, n, dx, a_list, dts, params, periodic=True, want_dt_next=True):
    """Advance on the GPU with the given dt sequence; returns (state numpy,
    dt_next list, stats dict list)."""
    torch = torch_mod()
    import paper_1301_4498_amd as nyx
    box = nyx.make_box(n, NG, dx)
    gdtype = torch.float64 if params.precision == nyx.NYX_FP64 else torch.float32
    U = to_dev(state)
    Uo = U.clone()
    G = to_dev(grav, gdtype)
    ws = aligned_ws(nyx.workspace_bytes(params, box))
    dtn = torch.zeros(1, dtype=torch.float64, device="cuda")
    st = torch.zeros(10, dtype=torch.int64, device="cuda")
    dt_next, stats = [], []
    for k in range(len(a_list) - 1):
        st.zero_()
        nyx.hydro_step(params, box, U, G, dts[k], a_list[k], a_list[k + 1], Uo,
                       dt_next=dtn if want_dt_next else None, stats=st, workspace=ws)
        if periodic:
            nyx.fill_ghosts_periodic(box, Uo)
        torch.cuda.synchronize()
        dt_next.append(float(dtn.item()))
        stats.append(nyx.stats_dict(st))
        U, Uo = Uo, U
    return U.cpu().numpy(), dt_next, stats


def rel_l1(a, b):
    """Relative L1 error per component of the valid region."""
    va = a[:, NG:-NG, NG:-NG, NG:-NG]
    vb = b[:, NG:-NG, NG:-NG, NG:-NG]
    return [float(np.abs(va[c] - vb[c]).sum() / max(np.abs(vb[c]).sum(), 1e-300))
            for c in range(a.shape[0])]
