"""The committed tile table that bench.py runs its grid with: it parses, it
names a compiled tile shape, and it covers the bench grid (129^3 nodes,
complex128)."""
import json
import os

import pytest

from paper_1705_08849_amd import devices as D

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TUNE = os.path.join(ROOT, "paper_1705_08849_amd", "tune_gfx950.json")
COMPILED = {(64, 8), (48, 8), (32, 8), (32, 16)}


def test_table_covers_the_bench_grid_with_a_compiled_shape():
    with open(TUNE) as f:
        t = json.load(f)
    assert t["arch"] == "gfx950"
    nx, ny, nz = D.plain_device_128(2).nodes
    hits = [e for e in t["entries"] if (e["nx"], e["ny"], e["nz"], e["dtype"]) == (nx, ny, nz, 0)]
    assert len(hits) == 1
    e = hits[0]
    assert (e["tx"], e["ty"]) in COMPILED
    assert 1 <= e["zc"] <= 128


@pytest.mark.gpu
def test_table_loads_into_the_library():
    from paper_1705_08849_amd import fit
    fit.tune_load(TUNE)
