"""The compiled-in tuning table is the autotuner's stored table: regenerating
it from autotune_table.json must give the committed kdt_tuning.inc, and every
stored shape must be a valid entry."""
import os

from paper_2609_18316_amd import autotune


def test_compiled_table_matches_the_stored_table(tmp_path):
    out = tmp_path / "kdt_tuning.inc"
    autotune.write_inc(autotune.load_table(), str(out))
    with open(autotune.INC) as f:
        assert f.read() == out.read_text()


def test_stored_entries_are_valid():
    table = autotune.load_table()
    assert table
    for name, e in table.items():
        d, l2, k, kind = autotune._parse_key(name)
        assert d in (2, 3, 4, 8, 16) and 0 <= l2 <= 31 and k >= 1
        assert 2 <= e["leaf_size"] <= 256 and e["queries_per_wave"] in (1, 64)
        assert autotune.key(1 << l2, d, k, kind) == name
