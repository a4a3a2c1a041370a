"""CPU checks of the tile table that dense rounds build over the
partition-tiled in-edges (the synchronous pull of Eq. sync): every in-edge in
exactly one tile, tiles inside their partition and under their cap, slots of
split partitions consecutive, and the launch order largest first within each
group. The table is host logic (daic_tile_table touches no device)."""
import math

import numpy as np
import pytest

NONE = 0xFFFFFFFF


@pytest.fixture(scope="module")
def daic():
    from paper_1710_05785_amd import daic as d

    d.lib()
    return d


def expected_caps(pstart, max_edges, group_parts, share_div):
    """The cap of every partition, as the header defines it."""
    n_part = len(pstart) - 1
    if not share_div:
        return [max(1024, max_edges)] * n_part
    gp = group_parts or n_part
    caps = []
    for p in range(n_part):
        g0 = p - p % gp
        g1 = min(n_part, g0 + gp)
        c = max(1024, (int(pstart[g1]) - int(pstart[g0])) // share_div)
        if max_edges:
            c = min(c, max(1024, max_edges))
        caps.append(c)
    return caps


def check_table(t, pstart, lb, max_edges, group_parts, share_div):
    pstart = [int(x) for x in pstart]
    n_part = len(pstart) - 1
    tp, te, ts, order = (t[k].astype(np.int64) for k in ("tile_part", "tile_e", "tile_slot", "order"))
    nt = tp.size
    assert te.size == nt + 1
    assert te[0] == pstart[0] and te[-1] == pstart[-1]
    assert np.all(np.diff(te) >= 0) and np.all(np.diff(tp) >= 0)
    caps = expected_caps(pstart, max_edges, group_parts, share_div)
    slot = 0
    n_split = 0
    for p in range(n_part):
        tiles = np.nonzero(tp == p)[0]
        size = pstart[p + 1] - pstart[p]
        assert tiles.size == max(1, math.ceil(size / caps[p])), p
        assert te[tiles[0]] == pstart[p] and te[tiles[-1] + 1] == pstart[p + 1]
        assert np.all(te[tiles + 1] - te[tiles] <= caps[p])
        if tiles.size == 1:
            assert ts[tiles[0]] == NONE
        else:
            n_split += 1
            assert list(ts[tiles]) == list(range(slot, slot + tiles.size))
            slot += tiles.size
    assert t["n_split"] == n_split and t["n_slots"] == slot
    # the launch order: a permutation, groups in order, largest work first in each
    assert sorted(order.tolist()) == list(range(nt))
    gp = group_parts or n_part
    work = (te[1:] - te[:-1]) + np.where(ts == NONE, 2 * (1 << lb), 0)
    groups = tp[order] // gp
    assert np.all(np.diff(groups) >= 0)
    for g in np.unique(groups):
        o = order[groups == g]
        w = work[o]
        assert np.all(np.diff(w) <= 0)
        ties = np.diff(w) == 0
        assert np.all(np.diff(o)[ties] > 0)  # equal work keeps tile order


def test_tile_table_hand_case(daic):
    # partition 0: 5,000 in-edges under a cap of 2,048 -> 2,048 + 2,048 + 904;
    # partition 1: empty, one tile; partition 2: 4,000 -> 2,048 + 1,952
    t = daic.tile_table([0, 5000, 5000, 9000], lb=10, max_edges=2048)
    assert t["tile_part"].tolist() == [0, 0, 0, 1, 2, 2]
    assert t["tile_e"].tolist() == [0, 2048, 4096, 5000, 5000, 7048, 9000]
    assert t["tile_slot"].tolist() == [0, 1, 2, NONE, 3, 4]
    assert (t["n_split"], t["n_slots"]) == (2, 5)
    # work: 2048, 2048, 904, 0 + 2 * 1024, 2048, 1952
    assert t["order"].tolist() == [0, 1, 3, 4, 5, 2]


def test_tile_table_small_caps_round_up(daic):
    # a cap below 1,024 counts as 1,024
    t = daic.tile_table([0, 3000], lb=8, max_edges=10)
    assert t["tile_e"].tolist() == [0, 1024, 2048, 3000]


@pytest.mark.parametrize("mode", ["cap", "share", "share_groups", "share_groups_cap"])
@pytest.mark.parametrize("n_part", [1, 7, 300])
def test_tile_table_invariants(daic, mode, n_part):
    rng = np.random.default_rng(1000 + n_part)
    sizes = (rng.pareto(1.2, n_part) * 3000).astype(np.int64)
    sizes[rng.random(n_part) < 0.1] = 0  # empty partitions
    pstart = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint32)
    lb = 12
    kw = {"cap": dict(max_edges=4096), "share": dict(share_div=64),
          "share_groups": dict(share_div=16, group_parts=4),
          "share_groups_cap": dict(share_div=8, group_parts=5, max_edges=3000)}[mode]
    t = daic.tile_table(pstart, lb, **kw)
    check_table(t, pstart, lb, kw.get("max_edges", 0), kw.get("group_parts", 0), kw.get("share_div", 0))


def test_tile_table_rejects_bad_input(daic):
    with pytest.raises(daic.DaicError, match="decreases"):
        daic.tile_table([0, 10, 5], lb=10, max_edges=2048)
    with pytest.raises(daic.DaicError, match="partition width"):
        daic.tile_table([0, 10], lb=7, max_edges=2048)
    with pytest.raises(daic.DaicError, match="max_edges or share_div"):
        daic.tile_table([0, 10], lb=10)
