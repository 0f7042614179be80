"""The tuning table shipped beside libdpg.so (paper_1711_00984_amd/tune_gfx950.json,
written by paper_1711_00984_amd/tune_table.py on a gfx950 GPU): well formed, every
row a valid schedule, and every space, order and precision of the quadrature path
covered.  dpg_tables_build loads it; the GPU tests run with it loaded."""
import json
import os

import pytest

from oracle import shapes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TABLE = os.path.join(ROOT, "paper_1711_00984_amd", "tune_gfx950.json")
SPACES = ("H1", "HCURL", "HDIV", "L2")


def nslab(space, p):
    return sum(r[2] for r in shapes.ranges(space, p))


@pytest.mark.skipif(not os.path.exists(TABLE), reason="no shipped tuning table")
def test_shipped_tune_table():
    d = json.load(open(TABLE))
    assert d["arch"] == "gfx950"
    assert d["fields"] == ["space", "p", "prec", "reduced", "size_class", "slab_group", "ms", "diag"]
    seen = set()
    for row in d["tune"]:
        sp, p, prec, red, sc, g, ms, diag = row
        assert sp in range(4) and 1 <= p <= 11 and prec in (0, 1) and red in (0, 1, 2)
        assert 0 <= sc <= 31 and ms > 0
        assert 1 <= g <= nslab(SPACES[sp], p), row
        assert diag in (-1, 0, 1)
        if red:
            assert diag == -1                       # the reduced paths have no diagonal schedule
        seen.add((sp, p, prec, red))
    for sp in range(4):
        for p in range(1, 12):
            for prec in (0, 1):
                assert (sp, p, prec, 0) in seen, (sp, p, prec)
