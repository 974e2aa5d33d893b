"""The C-ABI library loads on a machine without a GPU, exports every entry
point include/nyx_hydro.h declares, and rejects bad arguments on the host
before anything is enqueued (no compute calls here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def nyx():
    import paper_1301_4498_amd as nyx
    if not os.path.exists(nyx._lib.LIB_PATH):
        pytest.skip("HIP library not built")
    return nyx


def _declared():
    src = open(os.path.join(ROOT, "include", "nyx_hydro.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(nyx_\w+)\s*\(", src, re.M)))


def test_every_declared_symbol_is_exported(nyx):
    L = nyx.lib()
    names = _declared()
    assert len(names) >= 14
    for name in names:
        assert hasattr(L, name), name
    assert sorted(nyx._lib.exported_symbols()) == names


def test_defaults_and_status_strings(nyx):
    p = nyx.default_params()
    assert p.gamma == 5.0 / 3.0 and p.eta_dual == 1e-4 and p.riemann_maxiter == 20
    assert p.cfl == 0.5 and p.precision == nyx.NYX_FP64
    assert p.recon == nyx.NYX_RECON_PPM and p.grav_energy_form == 1
    assert p.riemann == nyx.NYX_RIEMANN_TWOSHOCK
    L = nyx.lib()
    assert L.nyx_status_string(0) == b"ok"
    assert b"overlap" in L.nyx_status_string(-4)


def test_workspace_bytes(nyx):
    p = nyx.default_params()
    b = nyx.make_box((8, 6, 4), 4, 0.1)
    P = 16 * 14 * 12
    E = 10 * 8 * 6
    al = lambda x: (x + 63) // 64 * 64
    # primitives, chi, edge states, then the Godunov states of the three
    # Riemann stages (5 values per face)
    elems = al(6 * P) + al(E) + al(30 * E) + al(15 * E) + al(30 * E) + al(15 * E)
    # CFL maximum, partial counters, one-entry box table, block prefixes, step constants
    header = 256 + 64 * 10 * 8 + 512 + 256 + 256
    assert nyx.workspace_bytes(p, b) == header + 8 * elems
    p.precision = nyx.NYX_MIXED
    assert nyx.workspace_bytes(p, b) == header + 4 * elems


def _step(nyx, p, b, sin=0x10000000, g=0x20000000, dt=1e-3, ao=0.5, an=0.51, sout=0x30000000,
          ws=0x40000000, wsb=1 << 40):
    L = nyx.lib()
    return L.nyx_hydro_step(ctypes.byref(p) if p is not None else None,
                            ctypes.byref(b) if b is not None else None, sin, g, dt, ao, an, sout,
                            None, None, ws, wsb, None)


def test_argument_errors(nyx):
    p = nyx.default_params()
    b = nyx.make_box((8, 8, 8), 4, 0.1)
    assert _step(nyx, None, b) == -1
    assert _step(nyx, p, None) == -1
    assert _step(nyx, p, b, sin=None) == -1
    assert _step(nyx, p, b, dt=0.0) == -3
    assert _step(nyx, p, b, dt=float("nan")) == -3
    assert _step(nyx, p, b, ao=-1.0) == -3
    assert _step(nyx, p, b, an=0.0) == -3
    # in/out overlap
    assert _step(nyx, p, b, sout=0x10000008) == -4
    # workspace too small / misaligned
    assert _step(nyx, p, b, wsb=1024) == -7
    assert _step(nyx, p, b, ws=0x40000010) == -7
    for bad in ((7, 8, 8), (8, 0, 8), (8, 8, -2)):
        assert _step(nyx, p, nyx.make_box(bad, 4, 0.1)) == -2
    assert _step(nyx, p, nyx.make_box((8, 8, 8), 3, 0.1)) == -2
    # padded cell count at or above 2^29 (32-bit byte offsets of FP64 arrays)
    assert _step(nyx, p, nyx.make_box((808, 808, 808), 4, 0.1)) == -2
    ws = ctypes.c_size_t()
    assert nyx.lib().nyx_workspace_bytes(ctypes.byref(p), ctypes.byref(nyx.make_box((800, 800, 792), 4, 0.1)),
                                         ctypes.byref(ws)) == 0
    assert _step(nyx, p, nyx.make_box((8, 8, 8), 4, 0.0)) == -3
    b2 = nyx.make_box((8, 8, 8), 4, 0.1)
    b2.comp_stride = 10
    assert _step(nyx, p, b2) == -2
    for field, val in (("gamma", 1.0), ("riemann_maxiter", 0), ("precision", 7), ("cfl", 0.0),
                       ("small_pres", 0.0), ("riemann", 5), ("recon", 2),
                       ("grav_energy_form", 0), ("grav_energy_form", 3),
                       ("mixed_riemann_stop", -1.0), ("mixed_riemann_stop", float("nan"))):
        q = nyx.default_params(**{field: val})
        assert _step(nyx, q, b) == -3, field


def test_learned_flux_argument_errors(nyx):
    b = nyx.make_box((8, 8, 8), 4, 0.1)
    # the learned flux exists in the FP32-mixed form only
    p = nyx.default_params(riemann=nyx.NYX_RIEMANN_LEARNED, learned_stages_mask=7)
    p.mlp_weights = 0x50000000
    assert _step(nyx, p, b) == -6
    p = nyx.default_params(precision=nyx.NYX_MIXED, riemann=nyx.NYX_RIEMANN_LEARNED,
                           learned_stages_mask=7)
    assert _step(nyx, p, b) == -1                     # no weights
    p.mlp_weights = 0x50000008
    assert _step(nyx, p, b) == -3                     # misaligned weights
    p.mlp_weights = 0x50000000
    p.learned_stages_mask = 0
    assert _step(nyx, p, b) == -3
    p.learned_stages_mask = 7
    p.mlp_resid_tol = -1.0
    assert _step(nyx, p, b) == -3
    L = nyx.lib()
    assert L.nyx_mlp_loss_grad(None, 1, 10, 5 / 3, 0.1, 1, 1, None) == -1
    assert L.nyx_mlp_loss_grad(0x1000, 0x2000, 10, 1.0, 0.1, 0x3000, 0x4000, None) == -3
    assert L.nyx_mlp_adam(0x1000, 0x2000, 0x3000, 0x4000, 0, 1e-3, 0.9, 0.999, 1e-8, None) == -3
    assert L.nyx_mlp_pack(0x1000, 0x2008, None) == -3
    assert L.nyx_batch_set_harvest(None, 1, 1, 10, 0.5, 0) == -1
    t = (ctypes.c_int * 7)()
    assert L.nyx_batch_set_tuning(None, t) == -1
    assert L.nyx_batch_get_tuning(None, t) == -1
    assert L.nyx_batch_autotune(None, 1, 1, 1, 0.5, 0.5, 2, None, 3, None, t, None) == -1


def test_batch_argument_errors(nyx):
    L = nyx.lib()
    p = nyx.default_params()
    boxes = (nyx.Box * 2)(nyx.make_box((8, 8, 8), 4, 0.1), nyx.make_box((7, 8, 8), 4, 0.1))
    mn, one = ctypes.c_size_t(), ctypes.c_size_t()
    assert L.nyx_batch_workspace_bytes(ctypes.byref(p), 2, boxes, ctypes.byref(mn), ctypes.byref(one)) == -2
    assert L.nyx_batch_workspace_bytes(ctypes.byref(p), 0, boxes, ctypes.byref(mn), ctypes.byref(one)) == -2
    good = (nyx.Box * 2)(nyx.make_box((8, 8, 8), 4, 0.1), nyx.make_box((16, 8, 8), 4, 0.1))
    assert L.nyx_batch_workspace_bytes(ctypes.byref(p), 2, good, ctypes.byref(mn), ctypes.byref(one)) == 0
    assert 0 < mn.value < one.value
    h = ctypes.c_void_p()
    # a workspace smaller than the largest box is rejected before any upload
    assert L.nyx_batch_create(ctypes.byref(p), 2, good, 0x40000000, 4096, None, ctypes.byref(h)) == -7
    assert L.nyx_hydro_step_batched(None, 1, 1, 1, 0.5, 0.5, 2, None, None, None) == -1
    # a plan is required before any ghost-source mode is looked at
    for mode in (-1, 0, 1, 5):
        assert L.nyx_batch_set_ghost_source(None, mode, 1, 1, 1) == -1
    assert L.nyx_batch_fill_ghosts(None, 0, 1, 1, 1, 0x10000000, None) == -1


def test_level_fill_planning_errors(nyx):
    # planning is host work: valid layouts plan, bad ones are refused
    L = nyx.lib()
    I = ctypes.c_int
    def plan(layout, dom, coarse=None):
        boxes = (nyx.Box * len(layout))(*[nyx.make_box(n, 4, 1.0) for n, _ in layout])
        lo = (I * (3 * len(layout)))(*[v for _, l in layout for v in l])
        d = (I * 3)(*dom)
        nb = ctypes.c_size_t(0)
        if coarse:
            cb = (nyx.Box * len(coarse))(*[nyx.make_box(n, 4, 2.0) for n, _ in coarse])
            clo = (I * (3 * len(coarse)))(*[v for _, l in coarse for v in l])
            return L.nyx_fill_plan_bytes(len(layout), boxes, lo, d, len(coarse), cb, clo,
                                         ctypes.byref(nb)), nb.value
        return L.nyx_fill_plan_bytes(len(layout), boxes, lo, d, 0, None, None, ctypes.byref(nb)), nb.value
    rc, nb = plan([((8, 8, 8), (0, 0, 0)), ((8, 8, 8), (8, 0, 0))], (16, 8, 8))
    assert rc == 0 and nb > 0
    # overlapping valid regions
    assert plan([((8, 8, 8), (0, 0, 0)), ((8, 8, 8), (4, 0, 0))], (16, 8, 8))[0] == -2
    # a box outside the domain
    assert plan([((8, 8, 8), (12, 0, 0))], (16, 8, 8))[0] == -2
    # open ghost cells without a coarse level (improper nesting)
    assert plan([((8, 8, 8), (4, 4, 4))], (24, 24, 24))[0] == -2
    # with a coarse level covering them it plans
    assert plan([((8, 8, 8), (4, 4, 4))], (24, 24, 24), coarse=[((12, 12, 12), (0, 0, 0))])[0] == 0
    # a coarse level with a hole under the fine box's ghost cells
    assert plan([((8, 8, 8), (4, 4, 4))], (24, 24, 24),
                coarse=[((6, 12, 12), (6, 0, 0))])[0] == -2
    # an odd domain
    assert plan([((8, 8, 8), (0, 0, 0))], (9, 8, 8))[0] == -2


def test_two_level_sync_planning_errors(nyx):
    # planning is host work: nested even layouts plan, bad ones are refused
    L = nyx.lib()
    I = ctypes.c_int

    def plan(fine, coarse, dom):
        fb = (nyx.Box * len(fine))(*[nyx.make_box(n, 4, 1.0) for n, _ in fine])
        flo = (I * (3 * len(fine)))(*[v for _, l in fine for v in l])
        cb = (nyx.Box * len(coarse))(*[nyx.make_box(n, 4, 2.0) for n, _ in coarse])
        clo = (I * (3 * len(coarse)))(*[v for _, l in coarse for v in l])
        d = (I * 3)(*dom)
        nb = ctypes.c_size_t(0)
        return L.nyx_sync_plan_bytes(len(fine), fb, flo, d, len(coarse), cb, clo, ctypes.byref(nb))

    whole = [((8, 8, 8), (0, 0, 0))]
    assert plan([((8, 8, 8), (4, 4, 4))], whole, (16, 16, 16)) == 0
    # an odd fine corner or extent
    assert plan([((8, 8, 8), (3, 4, 4))], whole, (16, 16, 16)) == -2
    assert plan([((8, 6, 7), (4, 4, 4))], whole, (16, 16, 16)) == -2
    # the coarse level does not hold the fine level's uncovered neighbours
    assert plan([((8, 8, 8), (4, 4, 4))], [((4, 8, 8), (2, 0, 0))], (16, 16, 16)) == -2
    # overlapping fine boxes
    assert plan([((8, 8, 8), (2, 2, 2)), ((8, 8, 8), (4, 4, 4))], whole, (16, 16, 16)) == -2
    # a fine box outside the domain
    assert plan([((8, 8, 8), (12, 4, 4))], whole, (16, 16, 16)) == -2
    assert L.nyx_batch_set_flux_register(None, None, 0, None) == -1
    assert L.nyx_reflux(None, None, None, 6, None) == -1


def test_gravity_entry_points_validate_before_launch(nyx):
    # every refusal below happens on the host, before anything is enqueued
    L = nyx.lib()
    I = ctypes.c_int
    dom = (I * 3)(16, 16, 16)
    nb = ctypes.c_size_t(0)
    assert L.nyx_poisson_workspace_bytes(dom, ctypes.byref(nb)) == 0 and nb.value > 16 ** 3 * 8
    for bad in ((15, 16, 16), (0, 16, 16), (16, 16, 1 << 17)):
        assert L.nyx_poisson_workspace_bytes((I * 3)(*bad), ctypes.byref(nb)) == -2
    assert L.nyx_poisson_workspace_bytes(None, ctypes.byref(nb)) == -1
    cyc, rel = ctypes.c_int(0), ctypes.c_double(0.0)
    fake = 0x10000000  # never dereferenced: every call below is refused first
    args = lambda **k: dict(dom=dom, dx=1 / 16, coef=1.0, rho=fake, state=None, box=None,
                            phi=fake, tol=1e-10, cyc=40, ws=fake, wsb=nb.value, **k)

    def solve(a):
        return L.nyx_poisson_solve(a["dom"], a["dx"], a["coef"], a["rho"], a["state"], a["box"],
                                   a["phi"], a["tol"], a["cyc"], a["ws"], a["wsb"], None,
                                   ctypes.byref(cyc), ctypes.byref(rel))
    L.nyx_poisson_workspace_bytes(dom, ctypes.byref(nb))
    a = args()
    a["dx"] = -1.0
    assert solve(a) == -3
    a = args()
    a["cyc"] = 0
    assert solve(a) == -3
    a = args()
    a["tol"] = float("nan")
    assert solve(a) == -3
    a = args()
    a["wsb"] = nb.value - 8
    assert solve(a) == -7
    a = args()
    a["ws"] = fake + 8  # misaligned
    assert solve(a) == -7
    a = args()
    a["rho"] = None
    assert solve(a) == -1
    a = args()
    a["state"] = fake  # a state without its box
    assert solve(a) == -1
    box = nyx.make_box((16, 16, 8), 4, 1 / 16)
    a = args()
    a["state"], a["box"] = fake, ctypes.byref(box)  # box does not cover the domain
    assert solve(a) == -2
    assert L.nyx_gravity_from_phi(dom, 1 / 16, fake, ctypes.byref(box), fake, 0, None) == -2
    good = nyx.make_box((16, 16, 16), 4, 1 / 16)
    assert L.nyx_gravity_from_phi(dom, 1 / 16, fake, ctypes.byref(good), fake, 7, None) == -3
    assert L.nyx_cic_deposit(fake, fake, -1, dom, 1 / 16, fake, None) == -3
    assert L.nyx_cic_deposit(fake, fake, 0, dom, 1 / 16, None, None) == -1
    assert L.nyx_cic_deposit(fake, fake, 0, dom, 1 / 16, fake, None) == 0  # nothing to do


def _noalloc(nyx, p, b, sin=0x10000000, g=0x20000000, dt=1e-3, ao=0.5, an=0.51, sout=0x30000000):
    L = nyx.lib()
    return L.nyx_hydro_step_noalloc(ctypes.byref(p) if p is not None else None,
                                    ctypes.byref(b) if b is not None else None, sin, g, dt, ao,
                                    an, sout, None, None, None)


def test_noalloc_step_validates_before_launch(nyx):
    # host-side checks only: every case returns before any GPU call
    p = nyx.default_params()
    b = nyx.make_box((8, 8, 8), 4, 0.1)
    assert _noalloc(nyx, None, b) == -1
    assert _noalloc(nyx, p, None) == -1
    assert _noalloc(nyx, p, b, sin=None) == -1
    assert _noalloc(nyx, p, b, dt=0.0) == -3
    assert _noalloc(nyx, p, b, sout=0x10000008) == -4
    assert _noalloc(nyx, p, nyx.make_box((7, 8, 8), 4, 0.1)) == -2
    # the scratch limit: the largest cube that fits, and the next even one
    cap = nyx.noalloc_max_bytes()
    assert cap == 64 << 20
    for prec in (nyx.NYX_FP64, nyx.NYX_MIXED):
        q = nyx.default_params(precision=prec)
        fits = [m for m in range(8, 200, 2)
                if nyx.workspace_bytes(q, nyx.make_box((m, m, m), 4, 0.1)) <= cap]
        big = nyx.make_box((fits[-1] + 2,) * 3, 4, 0.1)
        assert _noalloc(nyx, q, big) == -8
        assert nyx.lib().nyx_status_string(-8).decode().startswith("box needs more scratch")
    assert fits[-1] >= 48  # FP32-mixed holds the 48^3 boxes of the level workload
