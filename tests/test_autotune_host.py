"""Host logic of the solver autotuner: candidate grid and cache keys."""
import json

from paper_2401_06747_amd import autotune


def test_candidates_are_valid_parameter_sets():
    c = autotune.candidates()
    assert len(c) == (len(autotune.OVERLAPS) * len(autotune.LOCAL_ITERS) * len(autotune.COARSE_ITERS)
                      * len(autotune.SMALL_FROM) * len(autotune.ROBIN) * len(autotune.LOCAL_STOP))
    assert all(p.overlap % 2 == 0 and 2 <= p.overlap <= 16 for p in c)
    assert all(p.robin < 0 or 0 < p.robin <= 0.9 for p in c) and all(0 <= p.local_stop < 1 for p in c)
    # both the Dirichlet and the Robin boundary, and both local stopping rules, are tried
    assert {p.robin < 0 for p in c} == {True, False} and {p.local_stop > 0 for p in c} == {True, False}
    assert len({(p.overlap, p.local_iters, p.coarse_iters, p.small_from, p.robin, p.local_stop) for p in c}) == len(c)


def test_bucket_groups_similar_images():
    assert autotune.bucket((3, 1080, 1920), 0.05) == autotune.bucket((3, 1100, 1900), 0.052)
    assert autotune.bucket((3, 1080, 1920), 0.05) != autotune.bucket((1, 1080, 1920), 0.05)
    assert autotune.bucket((3, 1080, 1920), 0.05) != autotune.bucket((3, 2160, 3840), 0.05)
    assert autotune.bucket((3, 1080, 1920), 0.01) != autotune.bucket((3, 1080, 1920), 0.05)


def test_cache_is_read_back(tmp_path):
    p = tmp_path / "t.json"
    p.write_text(json.dumps({"k": {"params": {"overlap": 6, "local_iters": 4, "coarse_iters": 32}, "ms": 1.0}}))
    t = autotune.Autotuner(str(p))
    assert t.cache["k"]["params"]["overlap"] == 6
