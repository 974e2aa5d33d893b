"""MI355X-native comoving PPM gas step of Nyx (Almgren et al.).

Python binding of the C ABI in include/nyx_hydro.h.  Functions carry the C
names without the ``nyx_`` prefix and only marshal arguments: tensors are
passed by device pointer and the stream defaults to torch's current stream.
PyTorch is used only for device memory and streams.
"""
from __future__ import annotations

import ctypes

from . import _lib
from ._lib import (NYX_FP64, NYX_LAUNCH_FUSED, NYX_LAUNCH_PERSISTENT, NYX_LAUNCH_STAGED,
                   NYX_MIXED, NYX_RECON_PLM, NYX_RECON_PPM, NYX_RIEMANN_LEARNED,
                   NYX_RIEMANN_LINEARIZED, NYX_RIEMANN_TWOSHOCK, STATS_FIELDS, Box, NyxError,
                   Params, Stats, check, lib)

__all__ = ["Box", "Params", "Stats", "NyxError", "NYX_FP64", "NYX_MIXED", "NYX_LAUNCH_STAGED",
           "NYX_LAUNCH_PERSISTENT", "NYX_LAUNCH_FUSED", "NYX_RIEMANN_TWOSHOCK",
           "NYX_RIEMANN_LEARNED", "NYX_RIEMANN_LINEARIZED", "NYX_RECON_PPM", "NYX_RECON_PLM",
           "default_params", "make_box", "workspace_bytes", "estimate_dt",
           "hydro_step", "hydro_step_noalloc", "noalloc_max_bytes", "fill_ghosts_periodic", "Batch", "FillPlan", "SyncPlan", "cic_deposit", "PoissonSolver",
           "gravity_from_phi", "stats_dict"]


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def default_params(**kw) -> Params:
    p = Params()
    lib().nyx_default_params(ctypes.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


def make_box(n, ng: int = 4, dx: float = 1.0, state_off: int = 0, grav_off: int = 0,
             comp_stride: int | None = None, grav_stride: int | None = None) -> Box:
    nx, ny, nz = (int(x) for x in n)
    P = (nx + 2 * ng) * (ny + 2 * ng) * (nz + 2 * ng)
    b = Box()
    b.n[0], b.n[1], b.n[2] = nx, ny, nz
    b.ng = ng
    b.state_off = state_off
    b.grav_off = grav_off
    b.comp_stride = P if comp_stride is None else comp_stride
    b.grav_stride = P if grav_stride is None else grav_stride
    b.dx = dx
    return b


def workspace_bytes(params: Params, box: Box) -> int:
    out = ctypes.c_size_t(0)
    check("nyx_workspace_bytes", lib().nyx_workspace_bytes(ctypes.byref(params), ctypes.byref(box),
                                                           ctypes.byref(out)))
    return out.value


def estimate_dt(params, box, state, a, cfl, dt_out, workspace, stream=None) -> None:
    ws_bytes = workspace.numel() * workspace.element_size()
    check("nyx_estimate_dt", lib().nyx_estimate_dt(
        ctypes.byref(params), ctypes.byref(box), _ptr(state), a, cfl, _ptr(dt_out),
        _ptr(workspace), ws_bytes, _stream(stream)))


def hydro_step(params, box, state_in, grav, dt, a_old, a_new, state_out, dt_next=None,
               stats=None, workspace=None, stream=None) -> None:
    ws_bytes = workspace.numel() * workspace.element_size() if workspace is not None else 0
    check("nyx_hydro_step", lib().nyx_hydro_step(
        ctypes.byref(params), ctypes.byref(box), _ptr(state_in), _ptr(grav), float(dt),
        float(a_old), float(a_new), _ptr(state_out), _ptr(dt_next), _ptr(stats), _ptr(workspace),
        ws_bytes, _stream(stream)))


def hydro_step_noalloc(params, box, state_in, grav, dt, a_old, a_new, state_out, dt_next=None,
                       stats=None, stream=None) -> None:
    check("nyx_hydro_step_noalloc", lib().nyx_hydro_step_noalloc(
        ctypes.byref(params), ctypes.byref(box), _ptr(state_in), _ptr(grav), float(dt),
        float(a_old), float(a_new), _ptr(state_out), _ptr(dt_next), _ptr(stats), _stream(stream)))


def noalloc_max_bytes() -> int:
    out = ctypes.c_size_t(0)
    check("nyx_noalloc_max_bytes", lib().nyx_noalloc_max_bytes(ctypes.byref(out)))
    return out.value


def fill_ghosts_periodic(box, state, ncomp=6, stream=None) -> None:
    check("nyx_fill_ghosts_periodic", lib().nyx_fill_ghosts_periodic(
        ctypes.byref(box), _ptr(state), ncomp, _stream(stream)))


def stats_dict(t) -> dict:
    """Device nyx_stats block (a uint8/int64 tensor of 80 bytes) -> dict."""
    vals = t.view(dtype=__import__("torch").int64).cpu().tolist()
    return dict(zip(STATS_FIELDS, vals))


def tie_break_by_traffic(table, tune, traffic, tie=0.03):
    """Launch orders of a plan re-picked where counters are known: for each
    stage i in `traffic` ({i: HBM bytes per launch of each candidate}), the
    candidate with the least traffic among those whose time table[i][c] is
    within `tie` of the stage's fastest; other stages keep `tune`."""
    out = list(tune)
    for i, per_cand in traffic.items():
        fastest = min(table[i])
        near = [c for c in range(len(table[i])) if table[i][c] <= fastest * (1.0 + tie)]
        out[i] = min(near, key=lambda c: (per_cand[c], table[i][c]))
    return out


class Batch:
    """A batched plan (nyx_batch_*) over boxes in shared state/gravity buffers."""

    def __init__(self, params: Params, boxes, workspace, stream=None):
        self.params = params
        self.nbox = len(boxes)
        self._boxes = (Box * self.nbox)(*boxes)
        self.workspace = workspace
        h = ctypes.c_void_p(0)
        ws_bytes = workspace.numel() * workspace.element_size()
        check("nyx_batch_create", lib().nyx_batch_create(
            ctypes.byref(params), self.nbox, self._boxes, _ptr(workspace), ws_bytes,
            _stream(stream), ctypes.byref(h)))
        self.handle = h

    @staticmethod
    def workspace_bytes(params: Params, boxes):
        arr = (Box * len(boxes))(*boxes)
        mn, one = ctypes.c_size_t(0), ctypes.c_size_t(0)
        check("nyx_batch_workspace_bytes", lib().nyx_batch_workspace_bytes(
            ctypes.byref(params), len(boxes), arr, ctypes.byref(mn), ctypes.byref(one)))
        return mn.value, one.value

    @property
    def num_groups(self) -> int:
        return lib().nyx_batch_num_groups(self.handle)

    def estimate_dt(self, state, a, cfl, dt, stream=None):
        check("nyx_batch_estimate_dt", lib().nyx_batch_estimate_dt(
            self.handle, _ptr(state), a, cfl, _ptr(dt), _stream(stream)))

    def min_dt(self, dt, stream=None):
        check("nyx_batch_min_dt", lib().nyx_batch_min_dt(self.handle, _ptr(dt), _stream(stream)))

    def step(self, state_in, grav, dt, a_old, a_new, state_out, dt_next=None, stats=None,
             stream=None):
        check("nyx_hydro_step_batched", lib().nyx_hydro_step_batched(
            self.handle, _ptr(state_in), _ptr(grav), _ptr(dt), float(a_old), float(a_new),
            _ptr(state_out), _ptr(dt_next), _ptr(stats), _stream(stream)))

    def tuning(self):
        t = (ctypes.c_int * _lib.STAGES)()
        check("nyx_batch_get_tuning", lib().nyx_batch_get_tuning(self.handle, t))
        return list(t)

    def set_tuning(self, tune):
        t = (ctypes.c_int * _lib.STAGES)(*tune)
        check("nyx_batch_set_tuning", lib().nyx_batch_set_tuning(self.handle, t))

    def tuning_key(self, device_name: str = "") -> str:
        """Cache key of this plan's tuning: form, device and box-shape histogram."""
        import hashlib
        hist = {}
        for b in self._boxes:
            k = (b.n[0], b.n[1], b.n[2])
            hist[k] = hist.get(k, 0) + 1
        h = hashlib.sha1(repr(sorted(hist.items())).encode()).hexdigest()[:16]
        p = self.params
        return "%s|prec%d|riem%d|mask%d|nbox%d|groups%d|%s" % (
            device_name, p.precision, p.riemann, p.learned_stages_mask, self.nbox,
            self.num_groups, h)

    def autotune(self, state_in, grav, dt, a_old, a_new, state_out, dt_next=None, reps=3,
                 cache=None, stream=None, traffic=None, tie=0.03):
        """Pick each stage's launch order (nyx_batch_autotune).  With a cache
        file (JSON), a stored choice for the same key is applied without
        timing, and a new one is stored.  traffic: optional {stage index:
        [HBM bytes per launch of each candidate]} (measured counters); among
        the candidates whose time is within `tie` of a stage's fastest, the
        one with the least traffic is kept.  Returns (tune, ms or None)."""
        import json
        import os
        key = None
        if cache is not None:
            import torch
            key = self.tuning_key(torch.cuda.get_device_name())
            if os.path.exists(cache):
                with open(cache) as fh:
                    db = json.load(fh)
                if key in db:
                    self.set_tuning(db[key]["tune"])
                    return db[key]["tune"], None
        nst, nc = _lib.STAGES, _lib.TUNE_CANDIDATES
        ms = (ctypes.c_float * (nst * nc))()
        t = (ctypes.c_int * nst)()
        check("nyx_batch_autotune", lib().nyx_batch_autotune(
            self.handle, _ptr(state_in), _ptr(grav), _ptr(dt), float(a_old), float(a_new),
            _ptr(state_out), _ptr(dt_next), int(reps), ms, t, _stream(stream)))
        tune = list(t)
        table = [[round(float(ms[i * nc + c]), 4) for c in range(nc)] for i in range(nst)]
        if traffic:
            tune = tie_break_by_traffic(table, tune, traffic, tie)
            self.set_tuning(tune)
        if cache is not None:
            db = {}
            if os.path.exists(cache):
                with open(cache) as fh:
                    db = json.load(fh)
            db[key] = {"tune": tune, "ms": table}
            tmp = cache + ".tmp%d" % os.getpid()
            with open(tmp, "w") as fh:
                json.dump(db, fh, indent=1)
            os.replace(tmp, cache)
        return tune, table

    @property
    def launch_mode(self) -> int:
        m = ctypes.c_int(0)
        check("nyx_batch_get_launch_mode", lib().nyx_batch_get_launch_mode(self.handle,
                                                                           ctypes.byref(m)))
        return m.value

    def set_launch_mode(self, mode: int):
        check("nyx_batch_set_launch_mode", lib().nyx_batch_set_launch_mode(self.handle, int(mode)))

    def persistent_aborted(self, stream=None) -> bool:
        a = ctypes.c_int(0)
        check("nyx_batch_persistent_aborted", lib().nyx_batch_persistent_aborted(
            self.handle, ctypes.byref(a), _stream(stream)))
        return bool(a.value)

    def autotune_mode(self, state_in, grav, dt, a_old, a_new, state_out, reps=3, stream=None):
        """Keep the fastest launch mode (nyx_batch_autotune_mode); returns
        (mode, [staged ms, persistent ms, fused ms], -1 where not available)."""
        ms = (ctypes.c_float * 3)()
        m = ctypes.c_int(0)
        check("nyx_batch_autotune_mode", lib().nyx_batch_autotune_mode(
            self.handle, _ptr(state_in), _ptr(grav), _ptr(dt), float(a_old), float(a_new),
            _ptr(state_out), int(reps), ms, ctypes.byref(m), _stream(stream)))
        return m.value, [round(float(v), 4) for v in ms]

    def set_flux_register(self, sync, level, reg):
        """Feed a two-level sync plan's register (device FP64, 6 x faces) from
        every later step: level 0 for the coarse boxes, 1 for the fine boxes;
        reg None detaches it."""
        check("nyx_batch_set_flux_register", lib().nyx_batch_set_flux_register(
            self.handle, sync.handle if sync is not None else None, int(level), _ptr(reg)))
        self._sync = sync  # keep the sync plan's tables alive

    def fill_ghosts(self, state, mode=0, grid=(1, 1, 1), stream=None):
        check("nyx_batch_fill_ghosts", lib().nyx_batch_fill_ghosts(
            self.handle, mode, grid[0], grid[1], grid[2], _ptr(state), _stream(stream)))

    def set_ghost_source(self, mode=-1, grid=(1, 1, 1)):
        """Later steps take the input's ghost cells from their source cells
        (mode 0: each box periodic; 1: the boxes tile a periodic domain as
        `grid`) instead of reading them; -1 reads them again."""
        check("nyx_batch_set_ghost_source", lib().nyx_batch_set_ghost_source(
            self.handle, int(mode), int(grid[0]), int(grid[1]), int(grid[2])))

    def close(self):
        if self.handle is not None and self.handle.value:
            lib().nyx_batch_destroy(self.handle)
            self.handle = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class FillPlan:
    """Ghost fill of an AMR level (nyx_fill_plan_*, nyx_fill_level).  boxes:
    nyx_box list of the level (state offsets and strides into one FP64
    buffer); lo: per box the global index of valid cell (0, 0, 0); dom: the
    periodic domain; coarse: None or (cboxes, clo) of the level below."""

    def __init__(self, boxes, lo, dom, coarse=None, stream=None):
        import torch
        n = len(boxes)
        self._boxes = (Box * n)(*boxes)
        self._lo = (ctypes.c_int * (3 * n))(*[int(v) for b in lo for v in b])
        self._dom = (ctypes.c_int * 3)(*[int(v) for v in dom])
        if coarse is not None:
            cb, clo = coarse
            self._cb = (Box * len(cb))(*cb)
            self._clo = (ctypes.c_int * (3 * len(cb)))(*[int(v) for b in clo for v in b])
            nc = len(cb)
        else:
            self._cb, self._clo, nc = None, None, 0
        nbytes = ctypes.c_size_t(0)
        check("nyx_fill_plan_bytes", lib().nyx_fill_plan_bytes(
            n, self._boxes, self._lo, self._dom, nc, self._cb, self._clo, ctypes.byref(nbytes)))
        raw = torch.empty(nbytes.value + 256, dtype=torch.uint8, device="cuda")
        off = (-raw.data_ptr()) % 256
        self.workspace = raw[off:off + nbytes.value]
        h = ctypes.c_void_p(0)
        check("nyx_fill_plan_create", lib().nyx_fill_plan_create(
            n, self._boxes, self._lo, self._dom, nc, self._cb, self._clo,
            _ptr(self.workspace), nbytes.value, _stream(stream), ctypes.byref(h)))
        self.handle = h

    def counts(self):
        c, i = ctypes.c_longlong(0), ctypes.c_longlong(0)
        check("nyx_fill_plan_counts", lib().nyx_fill_plan_counts(self.handle, ctypes.byref(c),
                                                                 ctypes.byref(i)))
        return c.value, i.value

    def fill(self, state, coarse_state=None, ncomp=6, stream=None, coarse_new=None, theta=0.0):
        """coarse_new with theta: the coarse data interpolated in time (subcycling)."""
        check("nyx_fill_level_time", lib().nyx_fill_level_time(
            self.handle, _ptr(state), _ptr(coarse_state), _ptr(coarse_new), float(theta),
            int(ncomp), _stream(stream)))

    def close(self):
        if self.handle is not None and self.handle.value:
            lib().nyx_fill_plan_destroy(self.handle)
            self.handle = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SyncPlan:
    """Two-level synchronisation (nyx_sync_plan_*, nyx_reflux,
    nyx_average_down).  fine = (boxes, lo) of the fine level in the periodic
    domain dom; coarse = (cboxes, clo) of the level below (domain dom / 2)."""

    def __init__(self, fine, coarse, dom, stream=None):
        import torch
        fb, flo = fine
        cb, clo = coarse
        nf, nc = len(fb), len(cb)
        self._fb = (Box * nf)(*fb)
        self._flo = (ctypes.c_int * (3 * nf))(*[int(v) for b in flo for v in b])
        self._cb = (Box * nc)(*cb)
        self._clo = (ctypes.c_int * (3 * nc))(*[int(v) for b in clo for v in b])
        self._dom = (ctypes.c_int * 3)(*[int(v) for v in dom])
        nbytes = ctypes.c_size_t(0)
        check("nyx_sync_plan_bytes", lib().nyx_sync_plan_bytes(
            nf, self._fb, self._flo, self._dom, nc, self._cb, self._clo, ctypes.byref(nbytes)))
        raw = torch.empty(nbytes.value + 256, dtype=torch.uint8, device="cuda")
        off = (-raw.data_ptr()) % 256
        self.workspace = raw[off:off + nbytes.value]
        h = ctypes.c_void_p(0)
        check("nyx_sync_plan_create", lib().nyx_sync_plan_create(
            nf, self._fb, self._flo, self._dom, nc, self._cb, self._clo,
            _ptr(self.workspace), nbytes.value, _stream(stream), ctypes.byref(h)))
        self.handle = h

    def counts(self):
        """(interface faces, reflux cells, covered coarse cells)."""
        f, r, c = ctypes.c_longlong(0), ctypes.c_longlong(0), ctypes.c_longlong(0)
        check("nyx_sync_plan_counts", lib().nyx_sync_plan_counts(
            self.handle, ctypes.byref(f), ctypes.byref(r), ctypes.byref(c)))
        return f.value, r.value, c.value

    def register(self):
        """A zeroed flux register (6 x faces FP64 on the device)."""
        import torch
        return torch.zeros(6 * max(self.counts()[0], 1), dtype=torch.float64, device="cuda")

    def reflux(self, coarse_state, reg, ncomp=6, stream=None):
        check("nyx_reflux", lib().nyx_reflux(self.handle, _ptr(coarse_state), _ptr(reg),
                                             int(ncomp), _stream(stream)))

    def average_down(self, coarse_state, fine_state, ncomp=6, stream=None):
        check("nyx_average_down", lib().nyx_average_down(
            self.handle, _ptr(coarse_state), _ptr(fine_state), int(ncomp), _stream(stream)))

    def close(self):
        if self.handle is not None and self.handle.value:
            lib().nyx_sync_plan_destroy(self.handle)
            self.handle = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _dom(dom):
    return (ctypes.c_int * 3)(*[int(v) for v in dom])


def cic_deposit(pos, mass, dom, dx, rho, stream=None):
    """Add the cloud-in-cell density of particles (pos: device (3, np) FP64,
    mass: device (np,)) to rho (device, the domain's cells, x fastest);
    dom = (nx, ny, nz)."""
    np_ = int(mass.numel())
    check("nyx_cic_deposit", lib().nyx_cic_deposit(_ptr(pos), _ptr(mass), np_, _dom(dom),
                                                   float(dx), _ptr(rho), _stream(stream)))


class PoissonSolver:
    """Multigrid solve of the periodic 7-point Poisson problem on a domain of
    dom = (nx, ny, nz) cells (nyx_poisson_solve), with its own workspace."""

    def __init__(self, dom):
        import torch
        self.dom = tuple(int(v) for v in dom)
        nb = ctypes.c_size_t(0)
        check("nyx_poisson_workspace_bytes",
              lib().nyx_poisson_workspace_bytes(_dom(self.dom), ctypes.byref(nb)))
        raw = torch.empty(nb.value + 256, dtype=torch.uint8, device="cuda")
        off = (-raw.data_ptr()) % 256
        self.workspace = raw[off:off + nb.value]

    def solve(self, rho, phi, dx, coef, tol=1e-10, max_vcycles=50, state=None, box=None,
              stream=None):
        """phi (device) in: initial guess, out: solution.  Returns (V-cycles,
        relative residual)."""
        cyc, rel = ctypes.c_int(0), ctypes.c_double(0.0)
        check("nyx_poisson_solve", lib().nyx_poisson_solve(
            _dom(self.dom), float(dx), float(coef), _ptr(rho), _ptr(state),
            ctypes.byref(box) if box is not None else None, _ptr(phi), float(tol),
            int(max_vcycles), _ptr(self.workspace), self.workspace.numel(), _stream(stream),
            ctypes.byref(cyc), ctypes.byref(rel)))
        return cyc.value, rel.value

    def enqueue(self, rho, phi, dx, coef, vcycles, state=None, box=None, stream=None):
        """Exactly `vcycles` V-cycles, kernels only (no synchronisation)."""
        check("nyx_poisson_solve", lib().nyx_poisson_solve(
            _dom(self.dom), float(dx), float(coef), _ptr(rho), _ptr(state),
            ctypes.byref(box) if box is not None else None, _ptr(phi), 0.0, int(vcycles),
            _ptr(self.workspace), self.workspace.numel(), _stream(stream), None, None))


def gravity_from_phi(phi, dom, dx, box, grav, precision, stream=None):
    """g = -grad(phi) (centred) into every padded cell of `box` in grav."""
    check("nyx_gravity_from_phi", lib().nyx_gravity_from_phi(
        _dom(dom), float(dx), _ptr(phi), ctypes.byref(box), _ptr(grav), int(precision),
        _stream(stream)))
