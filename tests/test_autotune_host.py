"""Host logic of the tile autotuner: the table takes the fastest variant that
kept the bits, per degree and call site, and renders as a header the library
compiles."""
import re

from paper_2507_22195_amd import autotune


def _fake():
    var = [dict(TM=128, TN=64, KC=16), dict(TM=128, TN=128, KC=16), dict(TM=64, TN=64, KC=16)]
    t = lambda *ms: {str(i): {"ms": m, "same_bits": m is not None and m > 0} for i, m in enumerate(ms)}
    return {"device": "test", "variants": var, "degrees": {
        "1": {"n_macro": 8, "shape": [2, 2, 2], "sites": {"update": t(3.0, 2.0, 1.0), "schur": t(1.0, 2.0, 3.0)}},
        "2": {"n_macro": 8, "shape": [2, 2, 2], "sites": {"update": t(3.0, 2.5, -0.5), "schur": t(2.0, 1.0, 3.0)}},
        "3": {"n_macro": 8, "shape": [2, 2, 2], "sites": {"update": t(1.0, 2.0, 3.0), "schur": t(2.0, 3.0, 1.5)}}}}


def test_pick_takes_the_fastest_bit_identical_variant():
    table = autotune.pick(_fake())
    assert table[1] == {"update": 2, "schur": 0}
    # variant 2 at p = 2 is faster but changed the bits (same_bits False): refused
    assert table[2] == {"update": 1, "schur": 1}
    assert table[3] == {"update": 0, "schur": 2}


def test_rendered_header_holds_the_table():
    txt = autotune.render(_fake())
    rows = re.findall(r"\{(\d+), (\d+)\},\s+// p = (\d)", txt)
    assert [(int(a), int(b), int(p)) for a, b, p in rows] == [(2, 0, 1), (1, 1, 2), (0, 2, 3), (0, 0, 4)]
    assert "p = 4 (not swept)" in txt
    assert "kTileTable[5][2]" in txt and "#pragma once" in txt


def test_committed_table_is_well_formed():
    txt = open(autotune.TABLE).read()
    rows = re.findall(r"\{(\d+), (\d+)\},\s+// p = (\d)", txt)
    assert [int(p) for _, _, p in rows] == [1, 2, 3, 4]
