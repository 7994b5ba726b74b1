"""GPU test of inpaint_solve_noalloc (through the C ABI): the solve on the
library's fixed scratch array returns what inpaint_solve returns with a caller
workspace, bit for bit, on two calls in a row where the second image is smaller
(it runs on the scratch contents the first call left), and again after a warm
start; an image beyond the array is refused before any launch."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2401_06747_amd as hdi
from paper_2401_06747_amd import _lib
from workloads import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _tensors(inst):
    f = torch.tensor(inst.f, dtype=torch.float32, device=DEV).contiguous()
    m = torch.tensor(inst.mask, dtype=torch.uint8, device=DEV).contiguous()
    return f, m


def _noalloc(f, m, u0=None):
    """inpaint_solve_noalloc called through ctypes; returns (status, u, report)."""
    L = _lib.lib()
    C, H, W = f.shape
    u = torch.full(f.shape, float("nan"), dtype=torch.float64, device=DEV)
    rep = _lib.hdi_solve_report()
    p = _lib.hdi_solve_params()
    print(f"inpaint_solve_noalloc {C}x{H}x{W} warm={u0 is not None}", flush=True)
    st = L.inpaint_solve_noalloc(_lib.hdi_image(W, H, C), ctypes.c_void_p(m.data_ptr()),
                                 ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(u.data_ptr()),
                                 ctypes.c_void_p(u0.data_ptr() if u0 is not None else 0), ctypes.byref(p),
                                 ctypes.byref(rep), ctypes.c_void_p(torch.cuda.current_stream(DEV).cuda_stream))
    torch.cuda.synchronize()
    return st, u, rep


def test_two_calls_in_a_row_match_inpaint_solve():
    big = synth.config2(768, 1024, 3, 0.03, item=91)
    small = synth.config2(181, 263, 1, 0.05, item=92)
    L = _lib.lib()
    assert L.hdi_inpaint_workspace_bytes(_lib.hdi_image(1024, 768, 3)) <= L.hdi_noalloc_scratch_bytes()
    results = []
    for inst in (big, small):
        f, m = _tensors(inst)
        st, u, rep = _noalloc(f, m)
        assert st == _lib.HDI_OK, L.hdi_last_error()
        ref, rref = hdi.inpaint_solve(f, m)
        torch.cuda.synchronize()
        assert rref["status"] == 0
        assert torch.equal(u, ref), (inst.name, (u - ref).abs().max().item())
        assert rep.outer_iters == rref["outer_iters"] and rep.vcycles == rref["vcycles"]
        assert list(rep.rel_residual)[:f.shape[0]] == rref["rel_residual"]
        assert rep.ms > 0
        results.append((f, m, u))
    # a warm start from the big image's result, after the small call used the array
    f, m, u_big = results[0]
    st, u, rep = _noalloc(f, m, u0=u_big)
    ref, rref = hdi.inpaint_solve(f, m, u0=u_big)
    torch.cuda.synchronize()
    assert st == _lib.HDI_OK and rref["status"] == 0
    assert torch.equal(u, ref) and rep.outer_iters == rref["outer_iters"] == 0


def test_binding_and_errors():
    inst = synth.config2(64, 96, 3, 0.05, item=93)
    f, m = _tensors(inst)
    u, rep = hdi.inpaint_solve_noalloc(f, m)
    ref, _ = hdi.inpaint_solve(f, m)
    torch.cuda.synchronize()
    assert rep["status"] == 0 and torch.equal(u, ref)
    # an empty mask is the same error as for inpaint_solve
    with pytest.raises(hdi.HdiError) as ei:
        hdi.inpaint_solve_noalloc(f, torch.zeros_like(m))
    assert ei.value.status == _lib.HDI_ERR_EMPTY_MASK
    # 4K RGB needs more than the array holds: refused before any launch
    big = torch.zeros((3, 2160, 3840), dtype=torch.float32, device=DEV)
    bm = torch.ones((2160, 3840), dtype=torch.uint8, device=DEV)
    out = torch.full(big.shape, 7.0, dtype=torch.float64, device=DEV)
    with pytest.raises(hdi.HdiError) as ei:
        hdi.inpaint_solve_noalloc(big, bm, out=out)
    assert ei.value.status == _lib.HDI_ERR_WORKSPACE and "no-allocation" in str(ei.value)
    assert bool((out == 7.0).all())
