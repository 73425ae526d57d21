"""The cutoff tool's host logic: the crossover rule on synthetic
measurements, and its count of GEMV-T row splits against the library's
own plan (read through workspace sizes with the unsplit form disabled)."""
import ctypes

import pytest


def test_recommend_rules():
    from paper_2108_02025_amd.cutoffs import recommend

    def dots(cross):
        return [{"n": 1 << e, "bytes": 16 << e, "single_us": 1.0 if e <= cross else 3.0, "two_stage_us": 2.0}
                for e in range(8, 14)]
    res = {"dot_f64": dots(11), "dot_f32": dots(12), "dot2_f32": dots(10)}
    gt = [{"rows": 128 * k, "cols": 1024, "splits": k, "unsplit_us": 1.0 if k <= 3 else 5.0, "split_us": 2.0}
          for k in (1, 2, 3, 4, 5)]
    res["gemv_t_f64"], res["gemv_t_f32"] = gt, gt
    rec = recommend(res)
    assert rec["dot_small_bytes"] == 16 << 10      # the smallest crossover of the three
    assert rec["gemv_t_small_splits"] == 3
    gt2 = [dict(r, unsplit_us=5.0) if r["splits"] == 2 else r for r in gt]
    res["gemv_t_f32"] = gt2                         # one shape at 2 ways loses: nothing is replaced
    assert recommend(res)["gemv_t_small_splits"] == 0


@pytest.mark.parametrize("es,dt", [(8, 0), (4, 1)])
def test_split_count_matches_library_plan(es, dt):
    import os

    import paper_2108_02025_amd as sb
    from paper_2108_02025_amd.cutoffs import _splits
    if not os.path.exists(sb.lib_path):
        from paper_2108_02025_amd import build
        build.build(verbose=False)
    L = sb.load()
    h = ctypes.c_void_p()
    assert L.sb_handle_create(None, 0, None, ctypes.byref(h)) == 0
    try:
        assert L.sb_set_cutoff(h, 1, 0) == 0      # no unsplit form: the plain plan
        for rows in (64, 100, 128, 192, 256, 383, 512, 1024, 5000):
            for cols in (100, 128, 1024, 4096, 16384):
                ws = L.sb_workspace_bytes(h, 0, dt, 0, 1, rows, cols)
                lib = ws // (cols * es) if ws else 1
                assert _splits(rows, cols, es) == lib, (rows, cols)
    finally:
        L.sb_handle_destroy(h)
