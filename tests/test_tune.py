"""The autotuner's tile rule and its table (host logic, CPU only)."""
import json

import pytest

from paper_2312_07725_amd import tune


def test_select_tile_minimises_the_worst_slowdown():
    # tile 4 is fastest on the small mesh, tile 5 on the large one; tile 5 is
    # 1.25x off on the small mesh, tile 4 only 1.01x off on the large one
    per = {16: {1: 22.0, 4: 18.0, 5: 22.5}, 32: {1: 126.0, 4: 111.0, 5: 110.0}}
    t, w = tune.select_tile(per)
    assert t == 4 and w == pytest.approx(111.0 / 110.0)


def test_select_tile_only_common_tiles_and_ties_to_the_smaller():
    # tile 9 was timed on one mesh only: it cannot be chosen, but it is still
    # that mesh's fastest, against which the slowdown is measured
    per = {16: {1: 10.0, 2: 10.0, 9: 5.0}, 32: {1: 50.0, 2: 50.0}}
    assert tune.select_tile(per) == (1, 2.0)
    with pytest.raises(ValueError):
        tune.select_tile({16: {1: 1.0}, 32: {2: 1.0}})


def test_committed_table_follows_the_rule():
    """The tiles in the committed table are the rule's choice on the times it
    records, and fit the library's per-degree limits (14, 6, 3, 2)."""
    with open(tune.TILES_PATH) as fh:
        doc = json.load(fh)
    limits = {2: 14, 3: 6, 4: 3, 5: 2}
    for p, e in doc["tiles"].items():
        per = {int(k[len("all_us_"):]): {int(t): v for t, v in e[k].items()} for k in e if k.startswith("all_us_")}
        assert tune.select_tile(per)[0] == e["epb"]
        assert 1 <= e["epb"] <= limits[int(p)]
    for p, e in doc["ensemble_tiles"].items():
        assert 1 <= e["epb"] <= limits[int(p)]
    assert tune.load_tiles() == {int(p): e["epb"] for p, e in doc["tiles"].items()}
    assert tune.load_ensemble_tiles() == {int(p): e["epb"] for p, e in doc["ensemble_tiles"].items()}
