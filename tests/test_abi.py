"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and its host-only helpers follow the paper's conventions."""
import json
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hdi.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"^\s*typedef[^;]*;", "", src, flags=re.M)   # function-pointer types are not entry points
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def _lib():
    from paper_2401_06747_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libhdi.so not built")
    return _lib


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["inpaint_solve", "hdi_inpaint_workspace_bytes", "hdi_block_count", "hdi_status_string", "hdi_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    L = _lib().lib()
    for n in _declared():
        assert hasattr(L, n), n
    # the binding wraps exactly what the header declares
    assert sorted(_lib().exported_symbols()) == _declared()


def test_block_count_matches_paper():
    """Sec. 3.3: 32x32 blocks with overlap 6 give 36852 local problems for a 4K
    colour image on the finest level (3 channels)."""
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_numbers.json")))["oras_local_problems_4k_rgb"]
    from paper_2401_06747_amd import hdi_block_count
    _lib()
    n = hdi_block_count(g["width"], g["height"], g["overlap"]) * g["channels"]
    assert n == g["value"]
    assert hdi_block_count(32, 32, 6) == 1 and hdi_block_count(33, 1, 6) == 2


def test_workspace_query_and_status_strings():
    L = _lib()
    lib = L.lib()
    assert lib.hdi_inpaint_workspace_bytes(L.hdi_image(0, 5, 1)) == 0
    assert lib.hdi_inpaint_workspace_bytes(L.hdi_image(5, 5, 2)) == 0
    small = lib.hdi_inpaint_workspace_bytes(L.hdi_image(64, 64, 1))
    big = lib.hdi_inpaint_workspace_bytes(L.hdi_image(3840, 2160, 3))
    assert 0 < small < big
    # per pixel and channel: three FP32 level buffers (plus a fourth on coarse
    # levels, about 1/3 more in total) and one FP64 iterate copy
    assert big < 3840 * 2160 * 3 * (12 * 4 / 3 + 4 / 3 + 8) + 2 ** 24
    assert lib.hdi_status_string(2) == b"empty mask"


def test_argument_errors_need_no_gpu():
    """Bad shapes and null pointers are rejected before any HIP call."""
    import ctypes
    L = _lib()
    lib = L.lib()
    rep = L.hdi_solve_report()
    st = lib.inpaint_solve(L.hdi_image(4, 4, 2), None, None, None, None, None, 0, None, ctypes.byref(rep), None)
    assert st == L.HDI_ERR_ARG
    st = lib.inpaint_solve(L.hdi_image(4, 4, 1), None, None, None, None, None, 0, None, ctypes.byref(rep), None)
    assert st == L.HDI_ERR_ARG and b"non-null" in lib.hdi_last_error()
    p = L.hdi_solve_params(0.0, 0, 3, 0, 0, 0)   # odd overlap
    st = lib.inpaint_solve(L.hdi_image(4, 4, 1), ctypes.c_void_p(16), ctypes.c_void_p(16), ctypes.c_void_p(16),
                           None, None, 0, ctypes.byref(p), ctypes.byref(rep), None)
    assert st == L.HDI_ERR_ARG
    st = lib.inpaint_solve(L.hdi_image(4, 4, 1), ctypes.c_void_p(16), ctypes.c_void_p(16), ctypes.c_void_p(16),
                           None, None, 0, None, ctypes.byref(rep), None)
    assert st == L.HDI_ERR_WORKSPACE


def test_argument_errors_of_the_later_entry_points_need_no_gpu():
    """Voronoi initialisation, labels, jump-flooding densification, the CG flag
    and the MSE-gain stop validate their arguments before any HIP call."""
    import ctypes
    L = _lib()
    lib = L.lib()
    dev = ctypes.c_void_p(16)          # never dereferenced: every call below fails first
    img = L.hdi_image(8, 6, 1)
    assert lib.hdi_vinit_workspace_bytes(L.hdi_image(0, 6, 1)) == 0
    assert lib.hdi_vinit_workspace_bytes(img) > lib.hdi_inpaint_workspace_bytes(img)
    assert lib.hdi_labels_workspace_bytes(0, 5) == 0 and lib.hdi_labels_workspace_bytes(8, 6) > 0
    vrep = L.hdi_vinit_report()
    for bad in (L.hdi_vinit_params(3, 0, 1.0, 0, L.hdi_solve_params()),        # weighting
                L.hdi_vinit_params(2, 1001, 1.0, 0, L.hdi_solve_params()),     # max_iters
                L.hdi_vinit_params(2, 0, -1.0, 0, L.hdi_solve_params()),       # tau
                L.hdi_vinit_params(2, 0, 1.0, 8, L.hdi_solve_params())):       # flags
        assert lib.voronoi_init(img, dev, dev, dev, None, dev, 1 << 30, ctypes.byref(bad), ctypes.byref(vrep),
                                None) == L.HDI_ERR_ARG
    assert lib.voronoi_init(img, dev, dev, None, None, dev, 1 << 30, None, ctypes.byref(vrep), None) == L.HDI_ERR_ARG
    assert lib.voronoi_init(img, dev, dev, dev, None, dev, 16, None, ctypes.byref(vrep), None) == L.HDI_ERR_WORKSPACE
    d2 = ctypes.c_uint64(0)
    assert lib.hdi_voronoi_labels(8, 6, dev, dev, 3, ctypes.byref(d2), dev, 1 << 20, None) == L.HDI_ERR_ARG
    assert lib.hdi_voronoi_labels(8, 6, dev, dev, -2, ctypes.byref(d2), dev, 1 << 20, None) == L.HDI_ERR_ARG
    assert lib.hdi_voronoi_labels(8, 6, dev, dev, 0, ctypes.byref(d2), dev, 8, None) == L.HDI_ERR_WORKSPACE
    n = ctypes.c_int64(0)
    for part in (2, 8, 2 | L.HDI_PART_JFA):
        assert lib.densify_step(8, 6, dev, dev, 1, part, None, ctypes.byref(n), dev, 1 << 20, None) == L.HDI_ERR_ARG
    rep = L.hdi_solve_report()
    p = L.hdi_solve_params(0.0, 0, 0, 0, 0, 8, 0)    # unknown flag bit
    assert lib.inpaint_solve(img, dev, dev, dev, None, dev, 1 << 30, ctypes.byref(p), ctypes.byref(rep),
                             None) == L.HDI_ERR_ARG
    trep = L.hdi_tonal_report()
    tp = L.hdi_tonal_params(0.0, 0, 0, 0, 0, 0, 0, L.hdi_solve_params(), 1.5)   # mse_gain >= 1
    assert lib.tonal_optimize(img, dev, dev, dev, None, dev, 1 << 30, ctypes.byref(tp), ctypes.byref(trep),
                              None) == L.HDI_ERR_ARG


def test_lds_calibration_and_statistics_arguments_need_no_gpu():
    """The LDS calibration and the LDS statistics reject bad arguments before
    any HIP call; the statistics are host-side and read 0 after a reset."""
    import ctypes
    L = _lib()
    lib = L.lib()
    bw = ctypes.c_double(-1.0)
    sink = ctypes.c_void_p(16)   # never dereferenced: every call below fails first
    assert lib.hdi_lds_calibrate(0, sink, ctypes.byref(bw), None) == L.HDI_ERR_ARG
    assert lib.hdi_lds_calibrate((1 << 20) + 1, sink, ctypes.byref(bw), None) == L.HDI_ERR_ARG
    assert lib.hdi_lds_calibrate(16, None, ctypes.byref(bw), None) == L.HDI_ERR_ARG
    assert lib.hdi_lds_calibrate(16, sink, None, None) == L.HDI_ERR_ARG
    v = ctypes.c_double(-1.0)
    assert lib.hdi_stats_get_lds(8, ctypes.byref(v)) == L.HDI_ERR_ARG
    assert lib.hdi_stats_get_lds(-1, ctypes.byref(v)) == L.HDI_ERR_ARG
    assert lib.hdi_stats_get_lds(6, None) == L.HDI_ERR_ARG
    lib.hdi_stats_reset()
    assert lib.hdi_stats_get_lds(6, ctypes.byref(v)) == L.HDI_OK and v.value == 0.0


def test_noalloc_solve_refuses_images_beyond_its_scratch_without_a_gpu():
    """inpaint_solve_noalloc checks the image against its fixed scratch array
    (HDI_NOALLOC_SCRATCH_MB MiB per GPU) before any HIP call."""
    import ctypes
    L = _lib()
    lib = L.lib()
    src = open(HEADER).read()
    mb = int(re.search(r"#define HDI_NOALLOC_SCRATCH_MB (\d+)", src).group(1))
    assert lib.hdi_noalloc_scratch_bytes() == mb << 20
    # the sizes the header names as fitting do fit
    assert lib.hdi_inpaint_workspace_bytes(L.hdi_image(1024, 768, 3)) <= mb << 20
    assert lib.hdi_inpaint_workspace_bytes(L.hdi_image(1920, 1080, 1)) <= mb << 20
    rep = L.hdi_solve_report()
    p16 = ctypes.c_void_p(16)
    st = lib.inpaint_solve_noalloc(L.hdi_image(3840, 2160, 3), p16, p16, p16, None, None, ctypes.byref(rep), None)
    assert st == L.HDI_ERR_WORKSPACE and b"no-allocation" in lib.hdi_last_error()
    st = lib.inpaint_solve_noalloc(L.hdi_image(4, 4, 1), None, p16, p16, None, None, ctypes.byref(rep), None)
    assert st == L.HDI_ERR_ARG
    st = lib.inpaint_solve_noalloc(L.hdi_image(4, 4, 2), p16, p16, p16, None, None, ctypes.byref(rep), None)
    assert st == L.HDI_ERR_ARG
