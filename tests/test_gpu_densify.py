"""GPU parity of densify_step (through the C ABI) against the oracle's exact
reading of Alg. 1 (Sec. 4.1): given the same float32 error map, the new masks and
the added pixel lists must be identical, byte for byte."""
import numpy as np
import pytest
import torch

import paper_2401_06747_amd as hdi
from oracle import densify as od
from workloads import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _gpu_step(mask, err, n_add, partition):
    mt = torch.tensor(mask, dtype=torch.uint8, device=DEV).contiguous()
    et = torch.tensor(err, dtype=torch.float32, device=DEV).contiguous()
    added = hdi.densify_step(mt, et, n_add, partition)
    torch.cuda.synchronize()
    return mt.cpu().numpy(), added.cpu().numpy().astype(np.int64)


def _compare(mask, err, n_add, partition):
    part = "delaunay" if partition == hdi.DELAUNAY else "voronoi"
    ref_mask, ref_added, _ = od.densify_step(mask, err, n_add, part)
    m_gpu, a_gpu = _gpu_step(mask, err, n_add, partition)
    assert np.array_equal(a_gpu, ref_added), (a_gpu[:10], ref_added[:10], len(a_gpu), len(ref_added))
    assert np.array_equal(m_gpu, ref_mask)
    return a_gpu


@pytest.mark.parametrize("partition", [hdi.DELAUNAY, hdi.VORONOI])
@pytest.mark.parametrize("shape,count,n_add", [((40, 60), 12, 10), ((64, 64), 80, 50), ((97, 131), 150, 120),
                                                ((1, 90), 5, 4), ((70, 1), 4, 3), ((2, 2), 1, 3),
                                                ((33, 47), 1, 5), ((120, 200), 300, 1000)])
def test_random_masks(partition, shape, count, n_add):
    H, W = shape
    rng = np.random.default_rng(H * 1000 + W + count)
    m = np.zeros(H * W, np.uint8)
    m[rng.choice(H * W, min(count, H * W), replace=False)] = 1
    m = m.reshape(H, W)
    err = (rng.random((H, W)) * 50).astype(np.float32) ** 2
    err[m != 0] = 0
    # repeated values create ties that exercise the index rule
    err[rng.random((H, W)) < 0.2] = 7.0
    _compare(m, err, n_add, partition)


def test_regular_grid_mask_many_ties():
    """Seeds on a lattice make many equidistant pixels and cocircular quads."""
    H, W = 64, 80
    m = np.zeros((H, W), np.uint8)
    m[4::8, 4::8] = 1
    err = np.ones((H, W), np.float32)
    err[m != 0] = 0
    _compare(m, err, 40, hdi.DELAUNAY)
    _compare(m, err, 40, hdi.VORONOI)


def test_densification_loop_matches_oracle_at_every_step():
    """Config-3 style loop at reduced size: solve, error map, densify; the GPU
    error map is fed to both densify steps and the masks must stay identical."""
    inst = synth.config3(270, 480)
    f = torch.tensor(inst.f, dtype=torch.float32, device=DEV)
    mask = inst.mask.copy()
    sched = od.schedule(int(mask.sum()), int(0.04 * mask.size), 4)
    prev = int(mask.sum())
    for target in sched:
        mt = torch.tensor(mask, device=DEV)
        u, rep = hdi.inpaint_solve(f, mt)
        assert rep["status"] == 0
        err_t = hdi.error_map(u, f)
        err = err_t.cpu().numpy()
        # the map itself: FP64 sum over channels, one rounding (numpy adds in channel order)
        ref = ((u.cpu().numpy() - inst.f.astype(np.float32).astype(np.float64)) ** 2).sum(0).astype(np.float32)
        assert np.array_equal(err, ref)
        added = _compare(mask, err, target - prev, hdi.DELAUNAY)
        assert len(added) == target - prev
        mask[np.unravel_index(added, mask.shape)] = 1
        prev = target
    assert int(mask.sum()) == sched[-1]


def test_negative_zero_errors_tie_with_zero():
    """-0.0 is an accepted error value equal to 0: cells whose free pixels all
    carry zero error pick their smallest free index, whatever the sign bit."""
    H, W = 40, 52
    rng = np.random.default_rng(5)
    m = np.zeros(H * W, np.uint8)
    m[rng.choice(H * W, 30, replace=False)] = 1
    m = m.reshape(H, W)
    err = np.zeros((H, W), np.float32)
    err[rng.random((H, W)) < 0.3] = np.float32(-0.0)
    # a few cells with positive errors so the ranking has something to order
    err[rng.random((H, W)) < 0.02] = 3.0
    err[m != 0] = 0
    for partition in (hdi.DELAUNAY, hdi.VORONOI):
        _compare(m, err, 25, partition)


def test_errors():
    m = torch.zeros((8, 8), dtype=torch.uint8, device=DEV)
    e = torch.zeros((8, 8), dtype=torch.float32, device=DEV)
    with pytest.raises(hdi.HdiError) as ei:
        hdi.densify_step(m, e, 3)
    assert ei.value.status == 2
    m[2, 2] = 1
    with pytest.raises(hdi.HdiError):
        hdi.densify_step(m, e, 3, partition=7)
    # invalid error values are rejected before the mask changes
    for bad in (-1.0, float("nan"), float("inf")):
        e2 = e.clone()
        e2[5, 5] = bad
        before = m.clone()
        with pytest.raises(hdi.HdiError) as ei:
            hdi.densify_step(m, e2, 3)
        assert ei.value.status == 1
        assert torch.equal(m, before)


def test_error_map_rgb_bit_exact():
    rng = np.random.default_rng(11)
    u = rng.normal(100, 40, (3, 37, 91))
    f = rng.uniform(0, 255, (3, 37, 91)).astype(np.float32)
    e = hdi.error_map(torch.tensor(u, device=DEV), torch.tensor(f, device=DEV)).cpu().numpy()
    d = u - f.astype(np.float64)
    ref = ((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]).astype(np.float32)
    assert np.array_equal(e, ref)
