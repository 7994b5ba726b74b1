"""GPU parity of the spatial optimisation (Sec. 4, Alg. 1) through the C ABI:
the Laplacian-dithered initial mask equals the oracle's bit for bit, and every
densification step of the loop adds exactly the oracle's pixels for the error
map the GPU computed (each step's inputs come back through the step hook)."""
import numpy as np
import pytest
import torch

import paper_2401_06747_amd as hdi
from oracle import densify as od
from oracle import inpaint as oi
from oracle import spatial as osp
from workloads import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _inputs(H, W, C, item):
    f = synth.textured_image(H, W, C, 6, item)
    r = synth.rng_for(6, item, 3000).random((H, W))
    return f, r, torch.tensor(f, dtype=torch.float32, device=DEV), torch.tensor(r, device=DEV)


@pytest.mark.parametrize("shape,n0", [((3, 97, 130), 400), ((1, 270, 480), 650), ((3, 33, 1), 3), ((1, 1, 77), 5)])
def test_initial_mask_bit_exact(shape, n0):
    C, H, W = shape
    f, r, ft, rt = _inputs(H, W, C, sum(shape))
    m, count = hdi.initial_mask(ft, rt, n0)
    ref = osp.initial_mask(f.astype(np.float32), n0, r)
    assert np.array_equal(m.cpu().numpy(), ref)
    assert count == int(ref.sum())


def test_initial_mask_constant_image_is_uniform():
    H, W = 40, 50
    f = np.full((1, H, W), 77.0)
    r = synth.rng_for(6, 99, 3000).random((H, W))
    m, count = hdi.initial_mask(torch.tensor(f, dtype=torch.float32, device=DEV), torch.tensor(r, device=DEV), 100)
    ref = osp.initial_mask(f, 100, r)
    assert np.array_equal(m.cpu().numpy(), ref) and count == int(ref.sum())


@pytest.mark.parametrize("partition,t", [(hdi.DELAUNAY, 1.0), (hdi.VORONOI, 1.08)])
def test_loop_steps_match_oracle(partition, t):
    C, H, W, d, n = 3, 128, 192, 0.05, 6
    f, r, ft, rt = _inputs(H, W, C, 7)
    part = "delaunay" if partition == hdi.DELAUNAY else "voronoi"
    seen = []
    mask, u, rep = hdi.spatial_optimize(ft, rt, d, n_steps=n, t=t, partition=partition,
                                        hook=lambda k, m, e, a: seen.append((k, m, e, a)))
    n_target = int(np.floor(d * H * W))
    m0 = osp.initial_mask(f.astype(np.float32), osp.start_size(n_target, n), r)
    assert rep["initial_count"] == int(m0.sum())
    assert np.array_equal(seen[0][1], m0)
    sched = od.schedule(int(m0.sum()), n_target, n, t)
    assert len(seen) == n
    for k, (step, m_before, e, added) in enumerate(seen):
        assert step == k
        ref_mask, ref_added, _ = od.densify_step(m_before, e, sched[k] - int(m_before.sum()), part)
        assert np.array_equal(added.astype(np.int64), ref_added), k
        nxt = seen[k + 1][1] if k + 1 < n else mask.cpu().numpy()
        assert np.array_equal(nxt, ref_mask), k
    assert rep["final_count"] == n_target == int(mask.sum())
    ref_u = oi.inpaint(f.astype(np.float32).astype(np.float64), mask.cpu().numpy())
    assert oi.rel_l2(u.cpu().numpy(), ref_u).max() <= 1e-5


def test_error_maps_are_the_solutions_errors():
    """The error map each step sees is fp32 of the squared error of a solution
    of the inpainting system for the mask before that step. The solves run to
    rel-res 1e-10 here, so that the map is compared, not the solver's accuracy
    (at the default 1e-6 a solution may differ from the oracle's by up to the
    1e-5 solution bar, more than this pointwise bar on the map allows)."""
    C, H, W = 1, 96, 128
    f, r, ft, rt = _inputs(H, W, C, 8)
    seen = []
    hdi.spatial_optimize(ft, rt, 0.06, n_steps=3, solve=hdi.SolveParams(rel_tol=1e-10),
                         hook=lambda k, m, e, a: seen.append((m, e)))
    for m, e in seen:
        u = oi.inpaint(f.astype(np.float32).astype(np.float64), m)
        ref = osp.error_map(u, f.astype(np.float32))
        assert np.abs(e.astype(np.float64) - ref).max() <= 1e-5 * max(1.0, ref.max())


def test_errors():
    f, r, ft, rt = _inputs(20, 30, 1, 9)
    for kw in ({"density": 0.0}, {"density": 1.5}, {"density": 0.1, "n_steps": 0}, {"density": 0.1, "t": 0.0},
               {"density": 0.1, "partition": 2}, {"density": 0.1, "partition": 8}):
        with pytest.raises(hdi.HdiError):
            hdi.spatial_optimize(ft, rt, **kw)
