"""The quilt's tile choice, host logic only (no GPU): lfdpr_quilt_tile against
a model of the rule the header documents, written here from that text.  A
tile of rows x views takes rows * views * W * 8 + (W + H) * 4 + 16 bytes of
LDS; the automatic tile is 4 rows, else 2, else 1, as long as at least
min(8, views) views fit (for 1 row, any), with the views spread evenly over
the subsets; a batch's bands (items x ceil(H / rows)) may not exceed 8192."""
import itertools
import math

import pytest

from paper_2601_19901_amd import lfdpr


def lds(rows, views, W, H):
    return rows * views * W * 8 + (W + H) * 4 + 16


def model(W, H, V, n, max_lds, rows=0, views=0):
    def fits(r, v):
        return lds(r, v, W, H) <= max_lds and n * math.ceil(H / r) <= 8192

    if rows:
        r, v = min(rows, H), min(views, V)
        return (r, v) if fits(r, v) else None
    for r in (4, 2, 1):
        if r > H and r > 1:
            continue
        vmax = 0
        while vmax < V and fits(r, vmax + 1):
            vmax += 1
        if vmax >= min(8, V) or (r == 1 and vmax >= 1):
            subsets = math.ceil(V / vmax)
            return r, math.ceil(V / subsets)
    return None


@pytest.fixture(scope="module")
def built():
    import os
    if not os.path.exists(lfdpr.LIB_PATH):
        pytest.skip("liblfdpr.so not built")
    return lfdpr


def test_tiles_of_the_benchmark_rigs(built):
    assert built.quilt_tile(512, 512, 48) == (4, 8)        # display-1M
    assert built.quilt_tile(512, 512, 192) == (4, 9)       # display-4M-ss4
    assert built.quilt_tile(1024, 1024, 48) == (2, 8)      # display-1M-spatial2x
    assert built.quilt_tile(512, 512, 48, n_items=16) == (4, 8)   # batch16


def test_automatic_tiles_follow_the_documented_rule(built):
    n_cases = 0
    for W, H, V, n, mx in itertools.product((1, 7, 96, 512, 1024, 4096), (1, 3, 96, 512, 4096), (1, 8, 12, 48, 192, 1024),
                                           (1, 16, 256), (32768, 65536, 163840)):
        got = built.quilt_tile(W, H, V, n_items=n, max_lds=mx)
        assert got == model(W, H, V, n, mx), (W, H, V, n, mx, got)
        if got:
            r, v = got
            assert lds(r, v, W, H) <= mx and 1 <= r <= H and 1 <= v <= V
            n_cases += 1
    assert n_cases > 300


def test_requested_tiles_are_clipped_or_refused(built):
    # rows and views beyond the rig are clipped to it
    assert built.quilt_tile(96, 96, 12, rows=200, views=2) == (96, 2)
    assert built.quilt_tile(96, 96, 12, rows=3, views=50) == (3, 12)
    # a tile beyond the LDS is refused: 96 rows x 12 views x 96 px x 8 B
    assert built.quilt_tile(96, 96, 12, rows=96, views=12) is None
    # a batch whose bands exceed the lists: 16 x 512 fit, 17 x 512 do not
    assert built.quilt_tile(512, 512, 48, n_items=16, rows=1, views=8) == (1, 8)
    assert built.quilt_tile(512, 512, 48, n_items=17, rows=1, views=8) is None
    for args in ((0, 512, 48), (512, 0, 48), (512, 512, 0), (5000, 512, 48), (512, 512, 2000)):
        assert built.quilt_tile(*args) is None
    assert built.quilt_tile(512, 512, 48, n_items=0) is None
    assert built.quilt_tile(512, 512, 48, rows=4, views=0) is None
