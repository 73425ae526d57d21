"""The tuning table on the host: every configuration it hands out is one the
batched encoder accepts, for every width inside a bucket (a bucket spans
widths up to 2^0.5 times its centre, so binary64 rows wider than the
centre may need more x chunks than the centre's configuration has)."""
import numpy as np
import pytest

import paper_2108_02025_amd as sb
from paper_2108_02025_amd.tuner import TuningTable

DT = {"f64": 0, "f32": 1, "bf16": 2, "e4m3": 3}


@pytest.fixture(scope="module")
def table():
    t = TuningTable.load()
    if t is None:
        pytest.skip("no tuning table for this library version")
    return t


@pytest.mark.parametrize("kind", list(DT))
def test_tuned_configurations_are_valid_across_each_bucket(table, kind):
    L = sb.load()
    widths = sorted({*range(64, 8193, 97), 4097, 5792, 5793, 8192})
    for m in (64, 1000, 8192):
        for n in widths:
            cfg = table(kind, m, n)
            assert cfg is not None
            d = sb.sb_gemv_desc()
            d.dtype, d.m, d.n, d.lda = DT[kind], m, n, n
            d.A, d.x, d.c = 1 << 40, 1 << 41, 1 << 42
            d.scales = (1 << 43) if DT[kind] >= 2 else None
            d.group, d.rows_per_tile, d.split = cfg["group"], cfg["rows_per_tile"], cfg["split"]
            arr = (sb.sb_gemv_desc * 1)(d)
            assert L.sb_gemv_batched_table_bytes(arr, 1, None) != (1 << 64) - 1, (kind, m, n, cfg)


def test_bucket_split_raised_only_where_needed(table):
    # binary64 5000 columns falls in the 4096 bucket; its x needs two 32 KiB chunks
    assert table("f64", 1000, 5000)["split"] >= 2
    e = table.buckets["f32/10/12"]
    assert table("f32", 1000, 4096)["split"] == e["split"]
