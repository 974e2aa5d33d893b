"""Seeded synthetic inputs for the comoving gas step.

This module only draws random fields and packs them into the state layout; it
holds none of the step's arithmetic and is shared by the tests, the benchmark
and the oracle harness.  The paper's own workloads (Santa Barbara cluster and
cosmological initial conditions) are not available, so every input here is a
synthetic stand-in with the distributions listed per workload.

Conventions:
  * lognormal(mean m, sigma_ln s): ln X ~ N(ln m - s^2/2, s^2), so E[X] = m;
  * fields are white (independent per cell) unless smoothed;
  * k^-2 smoothing: a white Gaussian field is filtered by |k|^-1 in Fourier
    space (integer wavenumbers, k = 0 removed), transformed back and rescaled
    to zero mean and the requested standard deviation;
  * state (Sec. 3.2): U = (rho, a rho u, a^2 (p/(gamma-1) + rho |u|^2 / 2),
    a^2 p/(gamma-1)), component-major, x fastest, ghosts filled periodically.
Arrays: shape (ncomp, nz + 2 ng, ny + 2 ng, nx + 2 ng), float64.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

GAMMA = 5.0 / 3.0
NG = 4


def lognormal(rng: np.random.Generator, shape, mean: float, sigma_ln: float) -> np.ndarray:
    mu = np.log(mean) - 0.5 * sigma_ln * sigma_ln
    return np.exp(rng.normal(mu, sigma_ln, size=shape))


def smooth_k2(rng: np.random.Generator, shape, sigma: float) -> np.ndarray:
    """White Gaussian noise filtered to a k^-2 power spectrum, zero mean,
    standard deviation ``sigma``.  ``shape`` is (nz, ny, nx)."""
    w = rng.standard_normal(size=shape)
    fk = np.fft.rfftn(w)
    kz = np.fft.fftfreq(shape[0]) * shape[0]
    ky = np.fft.fftfreq(shape[1]) * shape[1]
    kx = np.fft.rfftfreq(shape[2]) * shape[2]
    k2 = kz[:, None, None] ** 2 + ky[None, :, None] ** 2 + kx[None, None, :] ** 2
    filt = np.zeros_like(k2)
    nz = k2 > 0
    filt[nz] = 1.0 / np.sqrt(k2[nz])
    f = np.fft.irfftn(fk * filt, s=shape, axes=(0, 1, 2))
    f -= f.mean()
    sd = f.std()
    return f * (sigma / sd) if sd > 0 else f


def pad_periodic(f: np.ndarray, ng: int = NG) -> np.ndarray:
    """(ncomp, nz, ny, nx) -> padded with periodic ghost cells."""
    return np.ascontiguousarray(np.pad(f, ((0, 0), (ng, ng), (ng, ng), (ng, ng)), mode="wrap"))


def fill_periodic_inplace(f: np.ndarray, ng: int = NG) -> None:
    """Refill the ghost cells of a padded field from its own valid cells."""
    valid = f[:, ng:-ng, ng:-ng, ng:-ng].copy()
    f[...] = pad_periodic(valid, ng)


def fill_outflow_inplace(f: np.ndarray, ng: int = NG, axis: int = 0) -> None:
    """Zero-gradient ghosts along one lab axis (0 = x), periodic on the others."""
    ax = 3 - axis
    valid = f[:, ng:-ng, ng:-ng, ng:-ng]
    pads = [(0, 0), (ng, ng), (ng, ng), (ng, ng)]
    wrap = np.pad(valid, [p if i != ax else (0, 0) for i, p in enumerate(pads)], mode="wrap")
    out = np.pad(wrap, [(0, 0) if i != ax else (ng, ng) for i in range(4)], mode="edge")
    f[...] = out


def conserved(rho: np.ndarray, u: np.ndarray, p: np.ndarray, a: float,
              gamma: float = GAMMA) -> np.ndarray:
    """Pack primitives (valid region, shapes (nz,ny,nx) and (3,nz,ny,nx)) into
    the six conserved components scaled with ``a``."""
    ke = 0.5 * rho * (u[0] ** 2 + u[1] ** 2 + u[2] ** 2)
    rei = p / (gamma - 1.0)
    return np.stack([rho, a * rho * u[0], a * rho * u[1], a * rho * u[2],
                     a * a * (rei + ke), a * a * rei])


@dataclass
class Workload:
    """One box (or a list of boxes) with its step schedule."""
    name: str
    n: tuple                      # (nx, ny, nz) of a single box
    dx: float
    a0: float
    a1: float
    steps: int
    cfl: float = 0.5
    gamma: float = GAMMA
    state: np.ndarray | None = None
    grav: np.ndarray | None = None
    extra: dict = field(default_factory=dict)

    def a_at(self, k: int) -> float:
        return self.a0 + (self.a1 - self.a0) * k / self.steps


def _box_fields_cfg1(rng, n, a):
    nx, ny, nz = n
    shape = (nz, ny, nx)
    rho = lognormal(rng, shape, 1.0, 0.5)
    u = rng.normal(0.0, 0.3, size=(3,) + shape)
    p = lognormal(rng, shape, 0.6, 0.3)
    g = rng.normal(0.0, 0.05, size=(3,) + shape)
    return conserved(rho, u, p, a), g


def _box_fields_cfg2(rng, n, a, gamma=GAMMA):
    nx, ny, nz = n
    shape = (nz, ny, nx)
    rho = lognormal(rng, shape, 1.0, 0.3)
    u = np.stack([smooth_k2(rng, shape, 0.5) for _ in range(3)])
    p = 0.6 * rho ** gamma
    g = rng.normal(0.0, 0.05, size=(3,) + shape)
    return conserved(rho, u, p, a, gamma), g


def config1(n: int = 32, seed: int = 1) -> Workload:
    """Single periodic 32^3 box, dx = 1/32; rho lognormal(1, 0.5), U_d ~ N(0,
    0.3^2), p lognormal(0.6, 0.3), g_d ~ N(0, 0.05^2); a 0.50 -> 0.505 over 10
    steps at CFL 0.5."""
    w = Workload("box32_plain", (n, n, n), 1.0 / n, 0.50, 0.505, 10)
    rng = np.random.default_rng(seed)
    U, g = _box_fields_cfg1(rng, w.n, w.a0)
    w.state, w.grav = pad_periodic(U), pad_periodic(g)
    return w


def config2(n: int = 256, seed: int = 2) -> Workload:
    """Single periodic 256^3 box, dx = 1/256; rho lognormal(1, 0.3), U k^-2
    smoothed with sigma 0.5, p = 0.6 rho^gamma, g ~ N(0, 0.05^2); a 0.25 -> 0.26
    over 20 steps."""
    w = Workload("box256_smooth", (n, n, n), 1.0 / n, 0.25, 0.26, 20)
    rng = np.random.default_rng(seed)
    U, g = _box_fields_cfg2(rng, w.n, w.a0)
    w.state, w.grav = pad_periodic(U), pad_periodic(g)
    return w


CFG3_EDGES = (16, 24, 32, 48, 64)


def config3_shapes(nbox: int = 4096, seed: int = 3):
    """Box extents of the batched AMR level: each axis drawn uniformly from
    {16, 24, 32, 48, 64}."""
    rng = np.random.default_rng(seed)
    return [tuple(int(x) for x in rng.choice(CFG3_EDGES, size=3)) for _ in range(nbox)]


def config3_box(b: int, n, a: float = 0.25):
    """Fields of box ``b`` of the batched level (config-2 distributions, seed
    3000 + b), padded with self-periodic ghosts."""
    rng = np.random.default_rng(3000 + b)
    U, g = _box_fields_cfg2(rng, n, a)
    return pad_periodic(U), pad_periodic(g)


def config5(n: int = 512, seed: int = 5) -> Workload:
    """Stress box: dx = 1/n; rho lognormal sigma_ln 2 clipped to +-ln 100 about
    the median; T/T_mean lognormal sigma_ln 1.5; p = rho T c0^2/gamma with
    c0 = 0.05; U k^-2 smoothed sigma 0.5, clipped to |U| <= 30 c; g ~ N(0,
    0.2^2); a 0.10 -> 0.11 over 10 steps."""
    w = Workload("box512_stress", (n, n, n), 1.0 / n, 0.10, 0.11, 10)
    rng = np.random.default_rng(seed)
    shape = (n, n, n)
    lnr = rng.normal(0.0, 2.0, size=shape)
    lnr = np.clip(lnr, -np.log(100.0), np.log(100.0))
    rho = np.exp(lnr)
    T = lognormal(rng, shape, 1.0, 1.5)
    c0 = 0.05
    p = rho * T * (c0 * c0 / GAMMA)
    u = np.stack([smooth_k2(rng, shape, 0.5) for _ in range(3)])
    c = np.sqrt(GAMMA * p / rho)
    umag = np.sqrt((u * u).sum(axis=0))
    scale = np.minimum(1.0, 30.0 * c / np.maximum(umag, 1e-300))
    u = u * scale
    g = rng.normal(0.0, 0.2, size=(3,) + shape)
    w.state, w.grav = pad_periodic(conserved(rho, u, p, w.a0)), pad_periodic(g)
    return w


def random_box(n, seed: int, a: float = 0.5, kind: int = 1):
    """A padded (state, grav) pair with config-1 (kind 1) or config-2 (kind 2)
    distributions on an arbitrary box extent n = (nx, ny, nz)."""
    rng = np.random.default_rng(seed)
    U, g = (_box_fields_cfg1 if kind == 1 else _box_fields_cfg2)(rng, n, a)
    return pad_periodic(U), pad_periodic(g)


def level_fields_torch(shapes, seed: int = 3, a: float = 0.25, gamma: float = GAMMA,
                       ng: int = NG, grav_dtype=None, device: str = "cuda"):
    """The batched AMR level (config-2 distributions per box) generated on the
    device with torch's seeded generator, for levels too large to draw with
    numpy in reasonable time.  Returns (state, grav, offsets) where state and
    grav are flat device tensors holding every padded box back to back and
    offsets[b] = (state_off, grav_off) in elements."""
    import torch
    gdt = grav_dtype or torch.float64
    sizes = [(n[0] + 2 * ng) * (n[1] + 2 * ng) * (n[2] + 2 * ng) for n in shapes]
    tot = sum(sizes)
    state = torch.empty(6 * tot, dtype=torch.float64, device=device)
    grav = torch.empty(3 * tot, dtype=gdt, device=device)
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    offs = []
    so = go = 0
    cache = {}
    for (nx, ny, nz), P in zip(shapes, sizes):
        shape = (nz, ny, nx)
        if shape not in cache:
            kz = torch.fft.fftfreq(nz, device=device) * nz
            ky = torch.fft.fftfreq(ny, device=device) * ny
            kx = torch.fft.rfftfreq(nx, device=device) * nx
            k2 = kz[:, None, None] ** 2 + ky[None, :, None] ** 2 + kx[None, None, :] ** 2
            filt = torch.where(k2 > 0, k2.clamp_min(1e-30).rsqrt(), torch.zeros_like(k2))
            cache[shape] = filt.to(torch.float64)
        filt = cache[shape]
        s_ln = 0.3
        rho = torch.exp(torch.randn(shape, generator=gen, device=device, dtype=torch.float64) * s_ln
                        - 0.5 * s_ln * s_ln)
        u = []
        for _ in range(3):
            w = torch.randn(shape, generator=gen, device=device, dtype=torch.float64)
            f = torch.fft.irfftn(torch.fft.rfftn(w) * filt, s=shape)
            f = f - f.mean()
            sd = f.std(unbiased=False)
            u.append(f * (0.5 / sd))
        p = 0.6 * rho ** gamma
        g = torch.randn((3,) + shape, generator=gen, device=device, dtype=torch.float64) * 0.05
        ke = 0.5 * rho * (u[0] ** 2 + u[1] ** 2 + u[2] ** 2)
        rei = p / (gamma - 1.0)
        U = torch.stack([rho, a * rho * u[0], a * rho * u[1], a * rho * u[2],
                         a * a * (rei + ke), a * a * rei])
        Up = torch.nn.functional.pad(U[None], (ng,) * 6, mode="circular")[0]
        gp = torch.nn.functional.pad(g[None], (ng,) * 6, mode="circular")[0]
        state[so:so + 6 * P] = Up.reshape(-1)
        grav[go:go + 3 * P] = gp.reshape(-1).to(gdt)
        offs.append((so, go))
        so += 6 * P
        go += 3 * P
    return state, grav, offs


def _k2_filter_torch(shape, device):
    """|k|^-1 filter (k = 0 removed) on the rfft grid of ``shape`` = (nz, ny, nx)."""
    import torch
    nz, ny, nx = shape
    kz = torch.fft.fftfreq(nz, device=device, dtype=torch.float64) * nz
    ky = torch.fft.fftfreq(ny, device=device, dtype=torch.float64) * ny
    kx = torch.fft.rfftfreq(nx, device=device, dtype=torch.float64) * nx
    k2 = kz[:, None, None] ** 2 + ky[None, :, None] ** 2 + kx[None, None, :] ** 2
    return torch.where(k2 > 0, k2.clamp_min(1e-30).rsqrt(), torch.zeros_like(k2))


def stress_fields_torch(n: int = 512, seed: int = 5, a: float = 0.10, gamma: float = GAMMA,
                        ng: int = NG, device: str = "cuda"):
    """The box512_stress fields of ``config5`` drawn on the device with torch's
    seeded generator (the numpy version of a 512^3 box takes minutes on the
    host).  Same distributions, different random stream.  Returns the padded
    state (6, n+2ng, n+2ng, n+2ng) and gravity (3, ...) as float64 device
    tensors."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    shape = (n, n, n)
    f64 = torch.float64

    def randn(sh):
        return torch.randn(sh, generator=gen, device=device, dtype=f64)

    lnr = (randn(shape) * 2.0).clamp_(-float(np.log(100.0)), float(np.log(100.0)))
    rho = torch.exp(lnr)
    del lnr
    s_t = 1.5
    T = torch.exp(randn(shape) * s_t - 0.5 * s_t * s_t)
    c0 = 0.05
    p = rho * T * (c0 * c0 / gamma)
    del T
    filt = _k2_filter_torch(shape, device)
    u = []
    for _ in range(3):
        f = torch.fft.irfftn(torch.fft.rfftn(randn(shape)) * filt, s=shape)
        f -= f.mean()
        f *= 0.5 / f.std(unbiased=False)
        u.append(f)
    del filt
    c = torch.sqrt(gamma * p / rho)
    umag = torch.sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2])
    scale = torch.clamp(30.0 * c / umag.clamp_min(1e-300), max=1.0)
    del c, umag
    u = [x * scale for x in u]
    del scale
    ke = 0.5 * rho * (u[0] ** 2 + u[1] ** 2 + u[2] ** 2)
    rei = p / (gamma - 1.0)
    del p
    state = torch.empty((6,) + tuple(s + 2 * ng for s in shape), dtype=f64, device=device)
    comps = [rho, a * rho * u[0], a * rho * u[1], a * rho * u[2], a * a * (rei + ke), a * a * rei]
    del u, ke, rei, rho
    for i, comp in enumerate(comps):
        state[i] = torch.nn.functional.pad(comp[None, None], (ng,) * 6, mode="circular")[0, 0]
        comps[i] = None
    grav = torch.empty((3,) + state.shape[1:], dtype=f64, device=device)
    for i in range(3):
        grav[i] = torch.nn.functional.pad((randn(shape) * 0.2)[None, None], (ng,) * 6,
                                          mode="circular")[0, 0]
    return state, grav


def split_patches(f, grid, ng: int = NG):
    """Cut a padded periodic domain (ncomp, Z + 2ng, Y + 2ng, X + 2ng) into
    gx * gy * gz padded patches of equal size, x fastest, each with its true
    neighbours as ghost cells.  Works on numpy arrays and torch tensors;
    returns views."""
    gx, gy, gz = grid
    mz = (f.shape[1] - 2 * ng) // gz
    my = (f.shape[2] - 2 * ng) // gy
    mx = (f.shape[3] - 2 * ng) // gx
    out = []
    for bz in range(gz):
        for by in range(gy):
            for bx in range(gx):
                out.append(f[:, bz * mz:bz * mz + mz + 2 * ng, by * my:by * my + my + 2 * ng,
                             bx * mx:bx * mx + mx + 2 * ng])
    return out


def join_valid(flat, grid, m, ncomp: int = 6, ng: int = NG):
    """Inverse of packing ``split_patches`` back to back: the valid cells of a
    flat patch buffer (equal m = (mx, my, mz) patches, x fastest) as one
    (ncomp, gz mz, gy my, gx mx) domain array (numpy or torch)."""
    gx, gy, gz = grid
    mx, my, mz = m
    v = flat.reshape(gz, gy, gx, ncomp, mz + 2 * ng, my + 2 * ng, mx + 2 * ng)
    v = v[:, :, :, :, ng:-ng, ng:-ng, ng:-ng]
    order = (3, 0, 4, 1, 5, 2, 6)
    v = v.transpose(*order) if isinstance(v, np.ndarray) else v.permute(*order)
    return v.reshape(ncomp, gz * mz, gy * my, gx * mx)
