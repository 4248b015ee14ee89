"""The stream-K work split of the 16-bit layer kernel, walked on the host by the library's own
plan code (fe_streamk_segments runs the walk the kernel runs; no device work).

For every padded size the schedules accept and several grid sizes it checks the properties the
kernel's correctness rests on:
* the (tile, K-block) iterations of the stream-K tiles are covered exactly once, and the leading
  data-parallel tiles not at all;
* every workgroup gets a non-empty range and publishes at most one partial (one slot each), as
  its first segment, before any of its waits;
* each tile has exactly one finishing segment; the workgroups it waits for (jlo .. j-1 of its
  group, all with smaller ids) are exactly the tile's publishers, and their blocks, in that
  order, are [0, kb0) without gaps.
"""
import os

import numpy as np
import pytest

from paper_2605_08523_amd import api


@pytest.fixture(scope="module", autouse=True)
def _lib():
    if not os.path.exists(api.LIB_PATH):
        pytest.fail("libfe.so is not built (python -m paper_2605_08523_amd.build)")
    api.lib()


def check_plan(np_, schedule, grid_offered):
    geom, _ = api.streamk_segments(np_, schedule, grid_offered, 0)
    T, ntiles, nk, dp, NG, grid = (geom[k] for k in ("T", "ntiles", "nk", "dp_tiles", "groups",
                                                    "grid"))
    tile = 256 if schedule == 1 else 128
    assert T == np_ // tile and ntiles == T * (T + 1) // 2
    assert 1 <= grid <= grid_offered and grid % NG == 0 and NG in (1, 8)
    assert 0 <= dp < ntiles
    per_tile = {}
    for w in range(grid):
        _, segs = api.streamk_segments(np_, schedule, grid_offered, w)
        assert len(segs) >= 1, f"workgroup {w} has an empty range"
        passes = segs[:, 0].tolist()
        assert passes == sorted(passes), "segments run in pass order"
        assert passes.count(0) <= 1, "one published partial per workgroup"
        assert passes.count(2) <= 1
        for (ps, t, kb0, kb1, jlo) in segs.tolist():
            assert dp <= t < ntiles and 0 <= kb0 < kb1 <= nk
            per_tile.setdefault(t, []).append((kb0, kb1, w, ps, jlo))
            if ps == 0:
                assert kb1 < nk, "a published partial never finishes its tile"
            else:
                assert kb1 == nk, "passes 1 and 2 finish their tile"
            if ps == 1:
                assert kb0 == 0
    assert sorted(per_tile) == list(range(dp, ntiles))
    for t, segs in per_tile.items():
        segs.sort()
        pos = 0
        for kb0, kb1, _, _, _ in segs:
            assert kb0 == pos, f"tile {t}: blocks covered with a gap or twice"
            pos = kb1
        assert pos == nk
        finishers = [s for s in segs if s[3] != 0]
        assert len(finishers) == 1
        kb0, _, w, ps, jlo = finishers[0]
        g, j = w % NG, w // NG
        pubs = sorted((s[2] // NG, s) for s in segs if s[3] == 0)
        if kb0 == 0:
            assert jlo == j and not pubs
            continue
        assert ps == 2 and 0 <= jlo < j
        assert [jj for jj, _ in pubs] == list(range(jlo, j)), f"tile {t}: waits != publishers"
        assert all(s[2] % NG == g for _, s in pubs), "publishers share the finisher's group"
        pos = 0
        for _, (b0, b1, _, _, _) in pubs:
            assert b0 == pos
            pos = b1
        assert pos == kb0
    return dict(geom)


@pytest.mark.parametrize("schedule,grids", [(2, (512, 608, 160, 16)), (1, (256, 304, 80, 8))])
def test_streamk_split_covers_and_hands_off(schedule, grids):
    tile = 256 if schedule == 1 else 128
    # every padded size from the smallest the library runs stream-K at (a 1536 workspace) up to
    # 8192, then larger sizes sparsely (the headline and the N = 16384 solve included)
    sizes = list(range(tile, 8192 + 1, tile)) + [12288, 16384]
    seen_groups = set()
    seen_dp = False
    for grid in grids:
        for np_ in sizes:
            if grid >= 512 and np_ > 8192 and schedule == 2 and np_ != 16384:
                continue
            g = check_plan(np_, schedule, grid)
            seen_groups.add(g["groups"])
            seen_dp |= g["dp_tiles"] > 0
    assert seen_groups == {1, 8}
    assert seen_dp == (schedule == 2)


def test_headline_plan():
    """N = 4096, 128 x 128 tiles, two workgroups per CU on 256 CUs: the 528 upper tiles are
    fewer than two rounds of 512, so all of them run stream-K, in 8 groups (one per XCD)."""
    g = check_plan(4096, 2, 512)
    assert g["ntiles"] == 528 and g["dp_tiles"] == 0 and g["groups"] == 8 and g["grid"] == 512


def test_argument_errors():
    lib = api.lib()
    import ctypes
    geom = (ctypes.c_int32 * 6)()
    cnt = ctypes.c_int32()
    assert lib.fe_streamk_segments(1000, 2, 512, 0, geom, None, 0, ctypes.byref(cnt)) == api.FE_ERR_ARG
    assert lib.fe_streamk_segments(1024, 3, 512, 0, geom, None, 0, ctypes.byref(cnt)) == api.FE_ERR_ARG
    assert lib.fe_streamk_segments(1024, 2, 0, 0, geom, None, 0, ctypes.byref(cnt)) == api.FE_ERR_ARG
    assert lib.fe_streamk_segments(1024, 2, 512, 9999, geom, None, 0, ctypes.byref(cnt)) == api.FE_OK
    assert cnt.value == 0
