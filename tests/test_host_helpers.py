"""Host-side input helpers: the patch split/join used by the patch-grid tests
and benchmark leg, and the stated distributions of the stress fields."""
import numpy as np

from paper_1301_4498_amd import synth


def test_split_join_roundtrip_numpy_and_torch():
    import torch
    rng = np.random.default_rng(0)
    dom = rng.normal(size=(6, 12, 8, 16))
    pad = synth.pad_periodic(dom)
    grid, m = (2, 1, 3), (8, 8, 4)
    parts = synth.split_patches(pad, grid)
    assert len(parts) == 6 and parts[0].shape == (6, 12, 16, 16)
    flat = np.concatenate([p.ravel() for p in parts])
    assert np.array_equal(synth.join_valid(flat, grid, m), dom)
    tparts = synth.split_patches(torch.from_numpy(pad), grid)
    tflat = torch.cat([p.reshape(-1) for p in tparts])
    assert torch.equal(synth.join_valid(tflat, grid, m), torch.from_numpy(dom))
    # a patch's ghost cells are its periodic neighbours' valid cells
    p = parts[1]  # bx = 1: x cells [8, 16) of the domain
    assert np.array_equal(p[:, 4:-4, 4:-4, -4:], dom[:, 0:4, 0:8, 0:4])


def test_stress_fields_distributions():
    n, g = 32, 5.0 / 3.0
    U, G = synth.stress_fields_torch(n=n, device="cpu")
    U, G = U.numpy(), G.numpy()
    v = U[:, 4:-4, 4:-4, 4:-4]
    rho = v[0]
    # density contrast at most 10^4 about the median (clipped at +-ln 100)
    assert rho.max() <= 100.0 * (1 + 1e-12) and rho.min() >= 0.01 * (1 - 1e-12)
    a = 0.10
    u = v[1:4] / (a * rho)
    p = v[5] / (a * a) * (g - 1.0)
    c = np.sqrt(g * p / rho)
    mach = np.sqrt((u * u).sum(axis=0)) / c
    assert mach.max() <= 30.0 * (1 + 1e-9)
    # total energy = internal + kinetic
    assert np.allclose(v[4], v[5] + 0.5 * a * a * rho * (u * u).sum(axis=0), rtol=1e-12)
    assert abs(G[:, 4:-4, 4:-4, 4:-4].std() - 0.2) < 0.01
    # ghosts are periodic copies
    assert np.array_equal(U[:, :4], U[:, n:n + 4])


def test_autotune_tie_break_by_traffic():
    from paper_1301_4498_amd import tie_break_by_traffic
    table = [[1.00, 1.02, 1.10, 1.01], [2.0, 1.5, 1.6, 3.0]]
    tune = [0, 1]
    # stage 0: candidates 0, 1, 3 are within 3% of the fastest; 3 moves the
    # fewest bytes; stage 1 has no record and keeps its fastest
    assert tie_break_by_traffic(table, tune, {0: [9e9, 8e9, 1e9, 5e9]}) == [3, 1]
    # equal traffic: the faster of the tied candidates
    assert tie_break_by_traffic(table, tune, {0: [5e9, 5e9, 5e9, 5e9]}) == [0, 1]
    # a much faster order is never traded for traffic
    assert tie_break_by_traffic(table, tune, {1: [1.0, 9e9, 1.0, 1.0]}) == [0, 1]
