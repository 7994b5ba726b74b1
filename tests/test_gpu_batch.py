"""GPU tests of hdi_solve_batch: uneven images in shared launches give, for every
image, bit-for-bit the result of the single-image solve, whatever else is in the
batch, and match the FP64 oracle (eq. inp-discrete-lsi)."""
import numpy as np
import pytest
import torch

import paper_2401_06747_amd as hdi
from oracle import inpaint as oi
from workloads import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _batch_items(k=8, seed=0):
    specs = synth.config4_specs(64)[:k]
    out = []
    for i, (H, W, C, d) in enumerate(specs):
        # reduced sizes (the full batch runs in the benchmark)
        H, W = max(33, H // 6), max(33, W // 6)
        f = synth.textured_image(H, W, C, 4, i)
        out.append((f, synth.gradient_mask(f, d)))
    return out


def _t(items):
    fs = [torch.tensor(f, dtype=torch.float32, device=DEV) for f, _ in items]
    ms = [torch.tensor(m, device=DEV) for _, m in items]
    return fs, ms


def test_batch_equals_single_solves_bitwise():
    items = _batch_items(8)
    fs, ms = _t(items)
    us, reps = hdi.solve_batch(fs, ms)
    for (f, m), u, rep in zip(zip(fs, ms), us, reps):
        u1, r1 = hdi.inpaint_solve(f, m)
        assert rep["status"] == 0 and r1["status"] == 0
        assert rep["outer_iters"] == r1["outer_iters"]
        assert torch.equal(u, u1)


def test_mixed_inpaint_and_tonal_jobs_equal_single_calls():
    """hdi_job.kind: inpainting and tonal jobs in one batch. The tonal jobs'
    inner solves run in the shared launches with the inpainting jobs; every
    result is bit-for-bit that of inpaint_solve or tonal_optimize alone."""
    items = _batch_items(6, seed=2)
    fs, ms = _t(items)
    kinds = [hdi.TONAL if i % 2 else hdi.INPAINT for i in range(len(fs))]
    tp = hdi.TonalParams(rel_tol=1e-7)
    outs, reps = hdi.solve_batch(fs, ms, kinds=kinds, tonal_params=tp)
    for f, m, k, out, rep in zip(fs, ms, kinds, outs, reps):
        assert rep["status"] == 0, rep
        if k == hdi.INPAINT:
            u1, r1 = hdi.inpaint_solve(f, m)
            assert torch.equal(out, u1) and rep["outer_iters"] == r1["outer_iters"]
        else:
            g1, r1 = hdi.tonal_optimize(f, m, params=tp)
            assert torch.equal(out, g1)
            assert rep["outer_iters"] == r1["outer_iters"] and rep["inner_solves"] == r1["inner_solves"]
            assert rep["mse_final"] == r1["mse_final"] and rep["rel_normal_residual"] <= 1e-7
    # a batch of tonal jobs only, with per-job parameters
    tps = [hdi.TonalParams(rel_tol=1e-7, mode=md) for md in (hdi.PCG_RAS, hdi.RAS, hdi.CGNR)]
    outs, reps = hdi.solve_batch(fs[:3], ms[:3], kinds=[hdi.TONAL] * 3, tonal_params=tps)
    for f, m, p, out in zip(fs[:3], ms[:3], tps, outs):
        assert torch.equal(out, hdi.tonal_optimize(f, m, params=p)[0])


def test_result_independent_of_batch_mix():
    items = _batch_items(6, seed=1)
    fs, ms = _t(items)
    full, _ = hdi.solve_batch(fs, ms)
    alone, _ = hdi.solve_batch(fs[2:3], ms[2:3])
    assert torch.equal(full[2], alone[0])
    rev, _ = hdi.solve_batch(fs[::-1], ms[::-1])
    for a, b in zip(full, rev[::-1]):
        assert torch.equal(a, b)


def test_batch_matches_oracle():
    items = _batch_items(4)
    fs, ms = _t(items)
    us, reps = hdi.solve_batch(fs, ms)
    for (f, m), u, rep in zip(items, us, reps):
        assert rep["status"] == 0
        err = oi.rel_l2(u.cpu().numpy(), oi.inpaint(f, m))
        assert err.max() <= 1e-5, (err, rep)
        assert oi.relres(u.cpu().numpy(), f, m).max() <= 1e-6 * 1.0001


def test_batch_with_per_job_params_and_tiny_images():
    rng = np.random.default_rng(4)
    items = []
    for (C, H, W) in [(1, 1, 40), (3, 17, 9), (1, 64, 64), (3, 45, 130)]:
        f = rng.uniform(0, 255, (C, H, W)).astype(np.float32).astype(np.float64)
        m = (rng.random((H, W)) < 0.1).astype(np.uint8)
        m[0, 0] = 1
        items.append((f, m))
    fs, ms = _t(items)
    params = [hdi.SolveParams(local_iters=6), hdi.SolveParams(), hdi.SolveParams(flags=1), hdi.SolveParams(coarse_iters=32)]
    us, reps = hdi.solve_batch(fs, ms, params=params)
    for (f, m), u, p in zip(zip(fs, ms), us, params):
        u1, _ = hdi.inpaint_solve(f, m, params=p)
        assert torch.equal(u, u1)


def test_empty_mask_in_batch_is_an_error():
    items = _batch_items(2)
    fs, ms = _t(items)
    ms[1] = torch.zeros_like(ms[1])
    with pytest.raises(hdi.HdiError) as ei:
        hdi.solve_batch(fs, ms)
    assert ei.value.status == 2


def test_batch_with_per_job_overlaps():
    items = _batch_items(4, seed=2)
    fs, ms = _t(items)
    params = [hdi.SolveParams(overlap=o, small_from=t) for o, t in ((2, 1), (4, -1), (6, 2), (16, 0))]
    us, reps = hdi.solve_batch(fs, ms, params=params)
    for f, m, u, p, rep in zip(fs, ms, us, params, reps):
        assert rep["status"] == 0
        u1, _ = hdi.inpaint_solve(f, m, params=p)
        assert torch.equal(u, u1)


def test_autotune_picks_a_converging_candidate_and_caches(tmp_path):
    from paper_2401_06747_amd import autotune
    f, m = _batch_items(1)[0]
    ft = torch.tensor(f, dtype=torch.float32, device=DEV)
    mt = torch.tensor(m, device=DEV)
    path = tmp_path / "tune.json"
    tuner = autotune.Autotuner(str(path), reps=1)
    p = tuner.params_for(ft, mt)
    key = lambda q: (q.overlap, q.local_iters, q.coarse_iters, q.small_from, q.robin, q.local_stop)  # noqa: E731
    assert key(p) in {key(c) for c in autotune.candidates()}
    u, rep = hdi.inpaint_solve(ft, mt, params=p)
    assert rep["status"] == 0
    assert oi.relres(u.cpu().numpy(), f, m).max() <= 1e-6 * 1.0001
    # a second tuner reads the cache instead of measuring again
    again = autotune.Autotuner(str(path)).params_for(ft, mt)
    assert key(again) == key(p)


def test_full_uneven_batch_equals_plain_solves():
    """The benchmark's 64-image batch at full size (512..2048 x 512..1152, gray and
    RGB, 1-10% masks): every image bit-for-bit equal to its plain solve, and the
    smallest one against the oracle."""
    from concurrent.futures import ThreadPoolExecutor
    specs = synth.config4_specs(64)
    with ThreadPoolExecutor(8) as ex:
        insts = list(ex.map(lambda a: synth.config4_item(*a), enumerate(specs)))
    fs = [torch.tensor(i.f, dtype=torch.float32, device=DEV) for i in insts]
    ms = [torch.tensor(i.mask, device=DEV) for i in insts]
    us, reps = hdi.solve_batch(fs, ms)
    assert all(r["status"] == 0 for r in reps)
    for f, m, u in zip(fs, ms, us):
        assert torch.equal(u, hdi.inpaint_solve(f, m)[0])
    k = min(range(64), key=lambda i: insts[i].f.size)
    err = oi.rel_l2(us[k].cpu().numpy(), oi.inpaint(insts[k].f, insts[k].mask))
    assert err.max() <= 1e-5, err
