"""The paper's Table 1 (flops and real loads per site of the clover hopping matrix) pins the
cost model that bench.py uses for its roofline: one spin-projected hop is 168 flops, the two
hermitian 6x6 clover products 552, and rebuilding the third row of a link from the first two
(row2 = conj(row0 x row1): three entries of two complex products and a difference) 42 flops,
saving 6 reals of load per link."""
import json
import os

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def table1():
    return json.load(open(os.path.join(HERE, "golden", "table1_flops.json")))["rows"]


def test_flop_model_matches_table1(table1):
    import bench

    # project (6 complex adds) + two SU(3) x colour-vector products (2 x (9 cmul + 6 cadd)) + rebuild (12 cadd)
    assert bench.HOP_FLOPS == 12 + 2 * (9 * 6 + 6 * 2) + 24
    # two 6x6 complex mat-vecs: 36 cmul + 30 cadd each
    assert bench.CLOVER_FLOPS == 2 * (36 * 6 + 30 * 2)
    assert 8 * bench.HOP_FLOPS + bench.CLOVER_FLOPS == table1["without_su3_reconstruction"]["flops"]
    recon_per_link = 3 * (2 * 6 + 2)
    assert 8 * recon_per_link == table1["with_su3_reconstruction"]["flops"] - table1["without_su3_reconstruction"]["flops"]


def test_load_model_matches_table1(table1):
    # 8 links per site in the hopping term; the compressed form drops one row of 3 complex numbers
    assert 8 * 6 == table1["without_su3_reconstruction"]["real_loads_stores"] - table1["with_su3_reconstruction"]["real_loads_stores"]
    for row in table1.values():
        assert abs(row["real_loads_stores"] / row["flops"] - row["real_per_flop"]) < 1e-4


def test_byte_per_flop_statement():
    t = json.load(open(os.path.join(HERE, "golden", "table1_flops.json")))
    r = t["rows"]["with_su3_reconstruction"]
    assert abs(4 * r["real_loads_stores"] / r["flops"] - t["required_byte_per_flop_sp_with_reconstruction"]) < 1e-3
