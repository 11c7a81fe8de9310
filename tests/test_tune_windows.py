"""The window tuner's header round trip (CPU): the table it writes is the
table it reads, in the layout the library compiles."""
import os

import paper_2501_15964_amd.tune_windows as tw


def test_header_round_trip(tmp_path):
    table = tw.read_header(tw.HEADER)
    assert len(table) == 3 * len(tw.LAYOUT_D)
    assert all(1 <= v <= 4096 for v in table.values())
    out = os.path.join(tmp_path, "tuned.hpp")
    tw.write_header(table, out)
    assert tw.read_header(out) == table
    changed = dict(table)
    changed[(10, 1)] = 7
    tw.write_header(changed, out)
    assert tw.read_header(out) == changed
    text = open(out).read()
    assert "constexpr int kTunedLayouts = %d;" % len(tw.LAYOUT_D) in text


def test_layouts_follow_the_row_dispatch():
    # one representative width per row layout, in increasing order, each
    # inside the range its name gives
    assert tw.LAYOUT_D == sorted(tw.LAYOUT_D)
    for d, name in zip(tw.LAYOUT_D, tw.LAYOUT_NAME):
        assert d <= int(name.split("<=")[1])
