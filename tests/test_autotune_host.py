"""Host logic of the autotuner: the table takes the fastest variant that kept
the bits, per degree and call site, and the fastest LU update depth whose
Ahat agreed with depth 1's, and renders as a header the library compiles."""
import re

from paper_2507_22195_amd import autotune


def _fake():
    var = [dict(TM=128, TN=64, KC=16), dict(TM=128, TN=128, KC=16), dict(TM=64, TN=64, KC=16)]
    t = lambda *ms: {str(i): {"ms": m, "same_bits": m is not None and m > 0} for i, m in enumerate(ms)}
    return {"device": "test", "variants": var, "degrees": {
        "1": {"n_macro": 8, "shape": [2, 2, 2], "sites": {"update": t(3.0, 2.0, 1.0), "schur": t(1.0, 2.0, 3.0)}},
        "2": {"n_macro": 8, "shape": [2, 2, 2], "sites": {"update": t(3.0, 2.5, -0.5), "schur": t(2.0, 1.0, 3.0)}},
        "3": {"n_macro": 8, "shape": [2, 2, 2], "sites": {"update": t(1.0, 2.0, 3.0), "schur": t(2.0, 3.0, 1.5)},
              "nblk": 14, "depths": {"1": {"ms": 10.0, "ok": True}, "2": {"ms": 9.0, "ok": True},
                                     "7": {"ms": 7.0, "ok": False}, "14": {"ms": 8.5, "ok": True}}}}}


def test_pick_takes_the_fastest_bit_identical_variant():
    table = autotune.pick(_fake())
    assert table[1] == {"update": 2, "schur": 0, "depth": 1}         # no depth sweep: depth 1
    # variant 2 at p = 2 is faster but changed the bits (same_bits False): refused
    assert table[2] == {"update": 1, "schur": 1, "depth": 1}
    # depth 7 is fastest but its Ahat left depth 1's: refused
    assert table[3] == {"update": 0, "schur": 2, "depth": 14}


def test_rendered_header_holds_the_table():
    txt = autotune.render(_fake())
    rows = re.findall(r"\{(\d+), (\d+)\},\s+// p = (\d)", txt)
    assert [(int(a), int(b), int(p)) for a, b, p in rows] == [(2, 0, 1), (1, 1, 2), (0, 2, 3), (0, 0, 4)]
    assert "p = 4 (not swept)" in txt
    assert "kTileTable[5][2]" in txt and "#pragma once" in txt
    assert re.search(r"kLuDepth\[5\] = \{1, 1, 1, 14, 1\}", txt)
    assert "depth  (14 blocks) 1:10.0, 2:9.0, 7:7.0!, 14:8.5" in txt


def test_committed_table_is_well_formed():
    txt = open(autotune.TABLE).read()
    rows = re.findall(r"\{(\d+), (\d+)\},\s+// p = (\d)", txt)
    assert [int(p) for _, _, p in rows] == [1, 2, 3, 4]
    d = re.search(r"kLuDepth\[5\] = \{1, (\d+), (\d+), (\d+), (\d+)\}", txt)
    assert d and all(int(x) >= 1 for x in d.groups())
