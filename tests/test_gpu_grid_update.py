"""The occupancy-grid estimator's EMA update on the GPU against the oracle."""
import numpy as np
import pytest
import torch

import oracle
import scenes
from gpu_util import dev, grid_spec, host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("res,L,jitter", [(4, 1, False), (32, 2, True), (128, 4, False)])
def test_grid_points(gpu_lib, res, L, jitter):
    n = L * res ** 3
    u = scenes.rng(62).random((n, 3)).astype(np.float32) if jitter else None
    g = grid_spec(gpu_lib, np.zeros(max(n // 32, 1), np.uint32), res, n_levels=L)
    got = host(gpu_lib.grid_points(g, None if u is None else dev(u)))
    ref = oracle.grid_points(res, n_levels=L, half_extent0=1.5, u=u)
    # binary32 evaluation of bmin + (i + u) * cell
    assert np.all(np.abs(got - ref) <= 4e-7 * (np.abs(ref) + 1.5 * 2 ** (L - 1)))


@pytest.mark.parametrize("n", [32, 4096 + 32, 4 * 128 ** 3])
def test_grid_ema(gpu_lib, n):
    g = scenes.rng(63)
    d0 = (g.exponential(0.02, n) * g.choice([0.0, 1.0], n, p=[0.3, 0.7])).astype(np.float32)
    s = (g.exponential(0.02, n) * g.choice([0.0, 1.0], n, p=[0.5, 0.5])).astype(np.float32)
    gamma, tau = 0.95, 0.01
    D = dev(d0)
    bits = torch.full((n // 32,), -1, dtype=torch.int32, device="cuda")
    gpu_lib.grid_ema(D, dev(s), gamma, tau, bits)
    rd, rocc = oracle.grid_ema(d0, s, np.float32(gamma), np.float32(tau))
    got = host(D)
    # two roundings of products and one of the sum, no cancellation (all >= 0)
    assert np.all(np.abs(got - rd) <= 3e-7 * np.abs(rd) + 1e-30)
    occ = scenes.unpack_bits(host(bits).view(np.uint32), n)
    band = np.abs(rd - tau) <= 1e-6 * tau
    assert np.array_equal(occ[~band], rocc[~band])
    assert 0.05 < rocc.mean() < 0.95


def test_estimator_update_then_march(gpu_lib):
    """OccupancyGrid.update with the analytic field at the cell centres (gamma = 0)
    gives the bits 1[sigma(centre) > tau]; the marcher then runs on them."""
    from paper_2305_04966_amd.pipeline import OccupancyGrid
    w = scenes.tiny(2048)
    res, tau = 32, 0.01
    bits = torch.zeros(res ** 3 // 32, dtype=torch.int32, device="cuda")
    grid = gpu_lib.GridSpec(bits, res, 1, (0.0, 0.0, 0.0), 1.5)
    est = OccupancyGrid(grid)
    fp = dev(w.fld.packed_params().astype(np.float32))

    def density(pts):
        n = pts.shape[0]
        z = torch.zeros(n, dtype=torch.float32, device="cuda")
        sig, _ = gpu_lib.blob_field(fp, w.fld.n_blobs, pts, torch.zeros_like(pts), z, z,
                                    fixed_count=1, want_rgb=False)
        return sig

    est.update(density, gamma=0.0, tau=tau)
    pts = oracle.grid_points(res, half_extent0=1.5)
    sref = oracle.field(pts, w.fld.packed_params())[0]
    occ = scenes.unpack_bits(host(bits).view(np.uint32), res ** 3)
    band = np.abs(sref - tau) <= 3e-4 * sref + 1e-6 * w.fld.peak  # binary32 field
    assert np.array_equal(occ[~band], (sref > tau)[~band])
    assert occ.any() and not occ.all()
    p = gpu_lib.march(grid, dev(w.rays_o), dev(w.rays_d), dt0=w.dt0)
    ref = oracle.march(w.rays_o, w.rays_d, host(bits).view(np.uint32), res, dt0=w.dt0)
    assert np.array_equal(host(p.packed_info), ref["packed_info"])
