"""FP64 CPU oracle of the Nyx comoving gas step -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It is a ctypes wrapper around
``oracle/nyx_oracle.c`` (plain C, built with ``-O2 -ffp-contract=off``) and
shares no code with the HIP library in ``paper_1301_4498_amd``.

What it computes is stated in ``nyx_oracle.c``: the unsplit PPM Godunov step
of Sec. 3.2 (Gas Dynamics) with the Step 2 predictor and Step 6 corrector and
dual-energy sync of Sec. 3.6, and the hydro CFL of Sec. 3.5.

Array convention: a field of ``ncomp`` components on a box of valid extent
(nx, ny, nz) with ``ng`` ghost cells is a C-contiguous float64 array of shape
``(ncomp, nz + 2 ng, ny + 2 ng, nx + 2 ng)``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libnyxoracle.so")
_SRC = os.path.join(_HERE, "nyx_oracle.c")
_MLP_SRC = os.path.join(_HERE, "mlp_oracle.c")
_FILL_SRC = os.path.join(_HERE, "fill_oracle.c")
_SYNC_SRC = os.path.join(_HERE, "sync_oracle.c")
_GRAV_SRC = os.path.join(_HERE, "gravity_oracle.c")

# Compiler line: plain IEEE FP64, no contraction, no fast-math.
CFLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-fPIC", "-shared", "-std=c11"]


def build(force: bool = True) -> str:
    """Compile the oracle shared library with gcc; returns its path."""
    if not force and os.path.exists(_SO):
        return _SO
    srcs = [_SRC, _MLP_SRC, _FILL_SRC, _SYNC_SRC, _GRAV_SRC]
    tmp = _SO + ".tmp%d" % os.getpid()
    cmd = ["gcc"] + CFLAGS + ["-o", tmp] + srcs + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _SO)
    return _SO


class _Params(ctypes.Structure):
    _fields_ = [
        ("gamma", ctypes.c_double),
        ("eta", ctypes.c_double),
        ("small_dens", ctypes.c_double),
        ("small_pres", ctypes.c_double),
        ("riemann_tol", ctypes.c_double),
        ("riemann_maxiter", ctypes.c_int32),
        ("recon", ctypes.c_int32),
        ("riemann", ctypes.c_int32),
        ("grav_form", ctypes.c_int32),
    ]


RECON_PPM, RECON_PLM = 0, 1
RIEMANN_TWOSHOCK, RIEMANN_LINEAR = 0, 1


class _Stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in (
        "nonfinite", "neg_dens", "neg_eint", "floor_hits", "trans_reverts",
        "sync_E_from_e", "riemann_iters", "riemann_calls")]


STATS_FIELDS = [f[0] for f in _Stats._fields_]


@dataclass
class Params:
    """Method parameters (Sec. 2.2: gamma = 5/3; Sec. 3.6 Step 6: eta = 1e-4)."""
    gamma: float = 5.0 / 3.0
    eta: float = 1e-4
    small_dens: float = 1e-20
    small_pres: float = 1e-20
    riemann_tol: float = 1e-14
    riemann_maxiter: int = 20
    recon: int = RECON_PPM          # Sec. 3.2: PPM, or PLM
    riemann: int = RIEMANN_TWOSHOCK  # Sec. 3.2: two-shock, or the linearised solver
    grav_form: int = 1               # Sec. 3.2: energy gravity term, form 1 or 2

    def c(self) -> _Params:
        return _Params(self.gamma, self.eta, self.small_dens, self.small_pres,
                       self.riemann_tol, int(self.riemann_maxiter), int(self.recon),
                       int(self.riemann), int(self.grav_form))


_lib = None
_D = ctypes.POINTER(ctypes.c_double)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        L = ctypes.CDLL(_SO)
        P = ctypes.POINTER(_Params)
        i = ctypes.c_int
        d = ctypes.c_double
        L.nyxo_estimate_dt.argtypes = [P, i, i, i, i, _D, d, d, d, _D]
        L.nyxo_estimate_dt.restype = i
        L.nyxo_hydro_step.argtypes = [P, i, i, i, i, _D, _D, d, d, d, d, _D,
                                      ctypes.POINTER(_Stats)]
        L.nyxo_hydro_step.restype = i
        L.nyxo_riemann.argtypes = [P, _D, _D, _D, _D, ctypes.POINTER(ctypes.c_int)]
        L.nyxo_riemann.restype = None
        L.nyxo_ppm_line.argtypes = [i, _D, _D, _D, _D]
        L.nyxo_ppm_line.restype = None
        L.nyxo_plm_line.argtypes = [i, _D, _D, _D, _D]
        L.nyxo_plm_line.restype = None
        _I32 = ctypes.POINTER(ctypes.c_int32)
        _I64 = ctypes.POINTER(ctypes.c_int64)
        L.nyxo_fill_level.argtypes = [i, _I32, _I32, _I64, i, _I32, i, _D, i, _I32, _I32, _I64, i,
                                      _D, _I64, _I64]
        L.nyxo_fill_level.restype = i
        L.nyxo_fill_level_time.argtypes = [i, _I32, _I32, _I64, i, _I32, i, _D, i, _I32, _I32,
                                           _I64, i, _D, _D, d, _I64, _I64]
        L.nyxo_fill_level_time.restype = i
        L.nyxo_hydro_step_faces.argtypes = [P, i, i, i, i, _D, _D, d, d, d, d, _D,
                                            ctypes.POINTER(_Stats), _D]
        L.nyxo_hydro_step_faces.restype = i
        L.nyxo_reflux_average_down.argtypes = [i, _I32, _I32, _I64, i, d, _D, _D, _I64, d,
                                               i, _I32, _I32, _I64, i, _I32, _D, i, _D, _I64,
                                               ctypes.c_int64, _D, i, _I64, _I64]
        L.nyxo_reflux_average_down.restype = i
        L.nyxo_cic_deposit.argtypes = [ctypes.c_long, _D, _D, _I32, d, _D]
        L.nyxo_cic_deposit.restype = i
        L.nyxo_cic_interp.argtypes = [ctypes.c_long, _D, _I32, d, _D, _D]
        L.nyxo_cic_interp.restype = i
        L.nyxo_gradient.argtypes = [_I32, d, _D, _D]
        L.nyxo_gradient.restype = i
        L.nyxo_ppm_interface.argtypes = [_D]
        L.nyxo_ppm_interface.restype = d
        L.nyxo_flatten_line.argtypes = [P, i, _D, _D, _D]
        L.nyxo_flatten_line.restype = None
        L.nyxo_flattening.argtypes = [P, i, i, i, i, _D, d, _D]
        L.nyxo_flattening.restype = i
        L.nyxo_trace_cell.argtypes = [P, i, _D, d, _D, _D, _D, d, d, d, d, _D, _D]
        L.nyxo_trace_cell.restype = i
        lg = ctypes.c_long
        L.nyxo_mlp_nparam.argtypes = []
        L.nyxo_mlp_nparam.restype = i
        L.nyxo_mlp_normalize.argtypes = [d, _D, lg, _D, _D]
        L.nyxo_mlp_normalize.restype = None
        L.nyxo_mlp_forward.argtypes = [_D, _D, lg, _D]
        L.nyxo_mlp_forward.restype = None
        L.nyxo_mlp_relu_pattern.argtypes = [_D, _D, lg]
        L.nyxo_mlp_relu_pattern.restype = ctypes.c_uint64
        L.nyxo_mlp_loss_grad.argtypes = [_D, _D, _D, lg, _D]
        L.nyxo_mlp_loss_grad.restype = d
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _dims(state: np.ndarray, ng: int):
    _, pz, py, px = state.shape
    return px - 2 * ng, py - 2 * ng, pz - 2 * ng


def estimate_dt(state: np.ndarray, ng: int, a: float, dx: float, cfl: float,
                params: Params | None = None) -> float:
    """Hydro CFL time step of Sec. 3.5 over the valid cells of one box."""
    params = params or Params()
    state = np.ascontiguousarray(state, dtype=np.float64)
    nx, ny, nz = _dims(state, ng)
    out = ctypes.c_double(0.0)
    rc = lib().nyxo_estimate_dt(ctypes.byref(params.c()), nx, ny, nz, ng,
                                _ptr(state), a, dx, cfl, ctypes.byref(out))
    if rc != 0:
        raise ValueError("nyxo_estimate_dt: bad arguments")
    return out.value


def face_flux_size(n) -> int:
    """Doubles in one box's face-flux block (layout of nyxo_hydro_step_faces)."""
    nx, ny, nz = n
    return 6 * ((nx + 1) * ny * nz + nx * (ny + 1) * nz + nx * ny * (nz + 1))


def face_flux_views(flux: np.ndarray, n):
    """Split a face-flux block into three arrays (6, nz', ny', nx') per direction."""
    nx, ny, nz = n
    out, pos = [], 0
    for d in range(3):
        shp = (6, nz + (d == 2), ny + (d == 1), nx + (d == 0))
        sz = int(np.prod(shp))
        out.append(flux[pos:pos + sz].reshape(shp))
        pos += sz
    return out


def hydro_step(state: np.ndarray, grav: np.ndarray, ng: int, dt: float,
               dx: float, a_old: float, a_new: float,
               params: Params | None = None, faces: bool = False):
    """One gas step.  Returns (new_state, stats dict), plus the final face
    fluxes (flat block, see face_flux_views) when faces is set.  Ghost cells
    of the returned array are copies of the input's (stale); refill before
    reuse."""
    params = params or Params()
    state = np.ascontiguousarray(state, dtype=np.float64)
    grav = np.ascontiguousarray(grav, dtype=np.float64)
    assert state.shape[0] == 6 and grav.shape == (3,) + state.shape[1:]
    nx, ny, nz = _dims(state, ng)
    out = state.copy()
    st = _Stats()
    flux = np.zeros(face_flux_size((nx, ny, nz))) if faces else None
    rc = lib().nyxo_hydro_step_faces(ctypes.byref(params.c()), nx, ny, nz, ng,
                                     _ptr(state), _ptr(grav), dt, dx, a_old, a_new,
                                     _ptr(out), ctypes.byref(st),
                                     _ptr(flux) if faces else None)
    if rc != 0:
        raise ValueError("nyxo_hydro_step: bad arguments")
    stats = {k: int(getattr(st, k)) for k in STATS_FIELDS}
    return (out, stats, flux) if faces else (out, stats)


def riemann(qL, qR, params: Params | None = None):
    """Riemann solve (two-shock, or the linearised solver per params) on
    rotated states (rho, u_n, u_t1, u_t2, p).
    Returns (godunov_state[5], {p, u, rhoL, rhoR}, iterations)."""
    params = params or Params()
    qL = np.ascontiguousarray(qL, dtype=np.float64)
    qR = np.ascontiguousarray(qR, dtype=np.float64)
    qg = np.zeros(5)
    star = np.zeros(4)
    it = ctypes.c_int(0)
    lib().nyxo_riemann(ctypes.byref(params.c()), _ptr(qL), _ptr(qR), _ptr(qg),
                       _ptr(star), ctypes.byref(it))
    return qg, dict(p=star[0], u=star[1], rhoL=star[2], rhoR=star[3]), it.value


def ppm_interface(q4) -> float:
    q4 = np.ascontiguousarray(q4, dtype=np.float64)
    return lib().nyxo_ppm_interface(_ptr(q4))


def ppm_line(q, chi=None):
    """Edge values (qm, qp) for cells 2..m-3 of a line; NaN elsewhere."""
    q = np.ascontiguousarray(q, dtype=np.float64)
    m = q.shape[0]
    chi = np.ones(m) if chi is None else np.ascontiguousarray(chi, dtype=np.float64)
    qm = np.full(m, np.nan)
    qp = np.full(m, np.nan)
    lib().nyxo_ppm_line(m, _ptr(q), _ptr(chi), _ptr(qm), _ptr(qp))
    return qm, qp


def plm_line(q, chi=None):
    """PLM edge values (qm, qp) for cells 2..m-3 of a line; NaN elsewhere."""
    q = np.ascontiguousarray(q, dtype=np.float64)
    m = q.shape[0]
    chi = np.ones(m) if chi is None else np.ascontiguousarray(chi, dtype=np.float64)
    qm = np.full(m, np.nan)
    qp = np.full(m, np.nan)
    lib().nyxo_plm_line(m, _ptr(q), _ptr(chi), _ptr(qm), _ptr(qp))
    return qm, qp


def flatten_line(p, u, params: Params | None = None):
    """Directional flattening coefficient for cells 3..m-4; NaN elsewhere."""
    params = params or Params()
    p = np.ascontiguousarray(p, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    chi = np.full(p.shape[0], np.nan)
    lib().nyxo_flatten_line(ctypes.byref(params.c()), p.shape[0], _ptr(p), _ptr(u),
                            _ptr(chi))
    return chi


def flattening(state: np.ndarray, ng: int, a: float, params: Params | None = None):
    """The step's flattening coefficient on the cells of [-1, n]^3 of a padded
    state (6, nz+2ng, ny+2ng, nx+2ng): shape (nz+2, ny+2, nx+2)."""
    params = params or Params()
    state = np.ascontiguousarray(state, dtype=np.float64)
    nx, ny, nz = _dims(state, ng)
    chi = np.full((nz + 2, ny + 2, nx + 2), np.nan)
    rc = lib().nyxo_flattening(ctypes.byref(params.c()), nx, ny, nz, ng, _ptr(state),
                               ctypes.c_double(a), _ptr(chi))
    if rc != 0:
        raise ValueError("nyxo_flattening: bad arguments")
    return chi


def trace_cell(d, qc, cc, qm, qp, g, kh, hdt_a=0.0, hda_a=0.0, pexp=0.0,
               params: Params | None = None):
    """Traced (left-face, right-face) lab-frame states of one cell."""
    params = params or Params()
    arr = [np.ascontiguousarray(x, dtype=np.float64) for x in (qc, qm, qp, g)]
    lo = np.zeros(5)
    hi = np.zeros(5)
    lib().nyxo_trace_cell(ctypes.byref(params.c()), d, _ptr(arr[0]), cc,
                          _ptr(arr[1]), _ptr(arr[2]), _ptr(arr[3]), kh, hdt_a,
                          hda_a, pexp, _ptr(lo), _ptr(hi))
    return lo, hi


# ---------------- learned-flux network (FP64 gradient oracle) ----------------

def mlp_nparam() -> int:
    return lib().nyxo_mlp_nparam()


def mlp_normalize(raw, gamma: float = 5.0 / 3.0):
    """Harvested face records (n, 15) -> network inputs (n, 10), targets (n, 5)."""
    raw = np.ascontiguousarray(raw, dtype=np.float64)
    n = raw.shape[0]
    x = np.zeros((n, 10))
    y = np.zeros((n, 5))
    lib().nyxo_mlp_normalize(gamma, _ptr(raw), n, _ptr(x), _ptr(y))
    return x, y


def mlp_forward(params, x):
    params = np.ascontiguousarray(params, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.zeros((x.shape[0], 5))
    lib().nyxo_mlp_forward(_ptr(params), _ptr(x), x.shape[0], _ptr(out))
    return out


def mlp_relu_pattern(params, x) -> int:
    params = np.ascontiguousarray(params, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    return int(lib().nyxo_mlp_relu_pattern(_ptr(params), _ptr(x), x.shape[0]))


def mlp_loss_grad(params, x, y):
    params = np.ascontiguousarray(params, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    g = np.zeros(params.shape[0])
    loss = lib().nyxo_mlp_loss_grad(_ptr(params), _ptr(x), _ptr(y), x.shape[0], _ptr(g))
    return loss, g


def fill_level(boxes, ng, dom, datas, coarse=None, ncomp=6, coarse_new=None, theta=0.0):
    """Ghost fill of one level (fill_oracle.c).  boxes: list of (n, lo) with
    n = (nx, ny, nz) and lo the global index of valid cell (0, 0, 0); datas:
    the boxes' padded arrays (ncomp, nz+2ng, ny+2ng, nx+2ng), filled in place
    (valid cells untouched); dom: the periodic domain (cells).  coarse: None
    or (cboxes, cng, cdatas) of the level below (ratio 2, ghosts filled).
    Returns (copied, interpolated) ghost-cell counts; raises if a ghost cell
    is covered by neither level.  coarse_new (the coarse boxes' arrays at the
    end of the coarse step) with theta in [0, 1]: the coarse data are
    interpolated in time, old + theta (new - old) (subcycling, Sec. 4.2)."""
    def pack(bxs, arrs):
        n3 = np.ascontiguousarray([list(n) for n, _ in bxs], dtype=np.int32).ravel()
        lo3 = np.ascontiguousarray([list(lo) for _, lo in bxs], dtype=np.int32).ravel()
        sizes = [a.size for a in arrs]
        off = np.ascontiguousarray(np.cumsum([0] + sizes[:-1]), dtype=np.int64)
        flat = np.ascontiguousarray(np.concatenate([np.ascontiguousarray(a, np.float64).ravel()
                                                    for a in arrs]))
        return n3, lo3, off, flat, sizes
    n3, lo3, off, flat, sizes = pack(boxes, datas)
    dom = np.ascontiguousarray(dom, dtype=np.int32)
    I32 = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    I64 = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    ncp, nip = ctypes.c_int64(0), ctypes.c_int64(0)
    cnew = None
    if coarse is not None:
        cb, cng, cd = coarse
        cn3, clo3, coff, cflat, _ = pack(cb, cd)
        args = (len(cb), I32(cn3), I32(clo3), I64(coff), cng, _ptr(cflat))
        if coarse_new is not None:
            cnew = pack(cb, coarse_new)[3]
    else:
        args = (0, None, None, None, 1, None)
    rc = lib().nyxo_fill_level_time(len(boxes), I32(n3), I32(lo3), I64(off), ng, I32(dom), ncomp,
                                    _ptr(flat), args[0], args[1], args[2], args[3], args[4],
                                    args[5], _ptr(cnew) if cnew is not None else None,
                                    float(theta), ctypes.byref(ncp), ctypes.byref(nip))
    if rc == -2:
        raise ValueError("a ghost cell is covered by neither level (improper nesting)")
    if rc != 0:
        raise ValueError("nyxo_fill_level: bad arguments")
    pos = 0
    for a, sz in zip(datas, sizes):
        a[...] = flat[pos:pos + sz].reshape(a.shape)
        pos += sz
    return ncp.value, nip.value


def reflux_average_down(cboxes, cng, cdx, cdatas, cfluxes, dt_c, fboxes, fng, dom, fdatas,
                        ffluxes, dt_f, ncomp=6):
    """Reflux and average-down of two levels (sync_oracle.c).  cboxes/fboxes:
    lists of (n, lo); cdatas: the coarse boxes' padded arrays, updated in
    place; cfluxes: per coarse box its step's face-flux block over dt_c;
    fdatas: the fine boxes' padded arrays after their substeps; ffluxes[s][b]:
    face-flux block of fine box b in substep s, over dt_f[s]; dom: the fine
    level's periodic domain.  Returns (interface faces, covered cells);
    raises on improper nesting."""
    I32 = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    I64 = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))

    def geom(bxs, arrs):
        n3 = np.ascontiguousarray([list(n) for n, _ in bxs], dtype=np.int32).ravel()
        lo3 = np.ascontiguousarray([list(lo) for _, lo in bxs], dtype=np.int32).ravel()
        sizes = [a.size for a in arrs]
        off = np.ascontiguousarray(np.cumsum([0] + sizes[:-1]), dtype=np.int64)
        flat = np.ascontiguousarray(np.concatenate([np.ascontiguousarray(a, np.float64).ravel()
                                                    for a in arrs]))
        return n3, lo3, off, flat, sizes

    def fluxcat(blocks):
        off = np.ascontiguousarray(np.cumsum([0] + [b.size for b in blocks[:-1]]), dtype=np.int64)
        return np.ascontiguousarray(np.concatenate(blocks), dtype=np.float64), off

    cn3, clo3, coff, cflat, csizes = geom(cboxes, cdatas)
    fn3, flo3, foff, fflat, _ = geom(fboxes, fdatas)
    cfl, cfl_off = fluxcat(list(cfluxes))
    subs = [fluxcat(list(f)) for f in ffluxes]
    stride = subs[0][0].size
    assert all(x[0].size == stride for x in subs)
    ffl = np.ascontiguousarray(np.concatenate([x[0] for x in subs]))
    ffl_off = subs[0][1]
    dtf = np.ascontiguousarray(dt_f, dtype=np.float64)
    dom = np.ascontiguousarray(dom, dtype=np.int32)
    nf, nc = ctypes.c_int64(0), ctypes.c_int64(0)
    rc = lib().nyxo_reflux_average_down(
        len(cboxes), I32(cn3), I32(clo3), I64(coff), cng, cdx, _ptr(cflat), _ptr(cfl),
        I64(cfl_off), dt_c, len(fboxes), I32(fn3), I32(flo3), I64(foff), fng, I32(dom),
        _ptr(fflat), len(subs), _ptr(ffl), I64(ffl_off), stride, _ptr(dtf), ncomp,
        ctypes.byref(nf), ctypes.byref(nc))
    if rc == -2:
        raise ValueError("improper nesting: a covered cell or its uncovered neighbour has no "
                         "coarse box")
    if rc != 0:
        raise ValueError("nyxo_reflux_average_down: bad arguments")
    pos = 0
    for a, sz in zip(cdatas, csizes):
        a[...] = cflat[pos:pos + sz].reshape(a.shape)
        pos += sz
    return nf.value, nc.value


# ---- gravity input path (gravity_oracle.c; Sec. 2.4, Sec. 3.4) ----
# Mesh fields of the periodic domain: arrays of shape (nz, ny, nx), no ghosts.

def _dom_of(shape):
    return np.ascontiguousarray([shape[2], shape[1], shape[0]], dtype=np.int32)


def cic_deposit(pos, mass, shape, dx, rho=None):
    """Cloud-in-cell comoving density of particles (pos: (3, np) x, y, z;
    mass: (np,)) on a periodic mesh of `shape` (nz, ny, nx); added to rho
    when given."""
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    mass = np.ascontiguousarray(mass, dtype=np.float64)
    out = np.zeros(shape) if rho is None else np.ascontiguousarray(rho, dtype=np.float64).copy()
    dom = _dom_of(shape)
    rc = lib().nyxo_cic_deposit(mass.size, _ptr(pos), _ptr(mass),
                                dom.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), dx, _ptr(out))
    if rc != 0:
        raise ValueError("nyxo_cic_deposit: bad arguments")
    return out


def cic_interp(pos, field, dx):
    """Cloud-in-cell value of a mesh field at particle positions (pins only)."""
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    field = np.ascontiguousarray(field, dtype=np.float64)
    out = np.zeros(pos.shape[1])
    dom = _dom_of(field.shape)
    rc = lib().nyxo_cic_interp(pos.shape[1], _ptr(pos),
                               dom.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), dx,
                               _ptr(field), _ptr(out))
    if rc != 0:
        raise ValueError("nyxo_cic_interp: bad arguments")
    return out


def gradient(phi, dx):
    """g = -(centred difference of phi) / (2 dx) per axis: (3, nz, ny, nx),
    components x, y, z."""
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    g = np.zeros((3,) + phi.shape)
    dom = _dom_of(phi.shape)
    rc = lib().nyxo_gradient(dom.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), dx, _ptr(phi),
                             _ptr(g))
    if rc != 0:
        raise ValueError("nyxo_gradient: bad arguments")
    return g


def laplacian7(phi, dx):
    """The standard 7-point Laplacian on the periodic mesh (Sec. 3.4)."""
    out = -6.0 * phi
    for ax in range(3):
        out = out + (np.roll(phi, 1, axis=ax) + np.roll(phi, -1, axis=ax))
    return out / (dx * dx)


def poisson_solve(rho, dx, coef):
    """The solution of the discrete periodic Poisson problem of Sec. 2.4 /
    Sec. 3.4: laplacian7(phi) = coef (rho - mean(rho)), phi of zero mean
    (the gauge of the periodic problem).  Exact up to rounding: the 7-point
    operator is diagonal in the discrete Fourier basis with eigenvalues
    sum_d (2 cos(2 pi k_d / n_d) - 2) / dx^2; the k = 0 mode is removed."""
    rho = np.asarray(rho, dtype=np.float64)
    f = coef * (rho - rho.mean())
    lam = np.zeros(rho.shape)
    for ax, n in enumerate(rho.shape):
        k = np.arange(n)
        e = (2.0 * np.cos(2.0 * np.pi * k / n) - 2.0) / (dx * dx)
        shp = [1, 1, 1]
        shp[ax] = n
        lam = lam + e.reshape(shp)
    fh = np.fft.fftn(f)
    lam[0, 0, 0] = 1.0
    ph = fh / lam
    ph[0, 0, 0] = 0.0
    return np.real(np.fft.ifftn(ph))
