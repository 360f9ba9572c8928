"""The XCD-aware tile orders of the split K build and the NT products
(xcd_strip_tile in kernels_lp.h), transcribed index for index: every
workgroup id of the launched grid maps to a distinct (row tile, strip) and
every tile is covered, for the launch shapes in use and ragged ones; each
XCD (id % 8) walks whole strips among the first 8 floor(nstrip/8).  Also the
banded XCD ranges of the two-body GEMM (k_gemm_tn_lds)."""
import pytest


def xcd_strip_tile(wg, n_rt, nstrip, deal=True):
    q8 = nstrip // 8 if deal else 0
    if wg < 8 * q8 * n_rt:
        li = wg // 8
        return li % n_rt, wg % 8 + 8 * (li // n_rt)
    i2 = wg - 8 * q8 * n_rt
    return i2 % n_rt, 8 * q8 + i2 // n_rt


def k_build_tile(wg, n_rt, n_full, n_ct, nseg, deal=True):
    """The K build's (row tile, column tile, segment): full column tiles in
    XCD-aware order, then the column tile with idle waves (if any)."""
    nf = n_rt * n_full * nseg
    if wg < nf:
        rt, strip = xcd_strip_tile(wg, n_rt, n_full * nseg, deal)
        return rt, strip % n_full, strip // n_full
    return (wg - nf) % n_rt, n_ct - 1, (wg - nf) // n_rt


@pytest.mark.parametrize("n_rt,n_full,n_ct,nseg", [
    (235, 16, 17, 19),      # N=128, 7500-row chunks, split BF16 (last column tile partly idle)
    (391, 25, 26, 31),      # N=160, 12500-row chunks
    (1, 1, 1, 1), (3, 1, 2, 2), (7, 3, 3, 5), (5, 8, 8, 1),
])
def test_k_build_tile_map_is_a_bijection(n_rt, n_full, n_ct, nseg):
    total = n_rt * n_full * nseg + (n_rt * nseg if n_full < n_ct else 0)
    for deal in (True, False):                       # dealt to XCDs, or plain order (large strips)
        tiles = {k_build_tile(w, n_rt, n_full, n_ct, nseg, deal) for w in range(total)}
        assert len(tiles) == total
        assert all(0 <= rt < n_rt and 0 <= ct < n_ct and 0 <= s < nseg for rt, ct, s in tiles)


@pytest.mark.parametrize("n_rt,nstrip", [(391, 489), (32, 17), (1, 1), (9, 8), (4, 23)])
def test_strip_order_bijection_and_xcd_affinity(n_rt, nstrip):
    seen, owner = set(), {}
    for w in range(n_rt * nstrip):
        rt, strip = xcd_strip_tile(w, n_rt, nstrip)
        assert 0 <= rt < n_rt and 0 <= strip < nstrip
        seen.add((rt, strip))
        if strip < 8 * (nstrip // 8):
            owner.setdefault(strip, set()).add(w % 8)
    assert len(seen) == n_rt * nstrip
    assert all(len(x) == 1 for x in owner.values())     # a dealt strip stays on one XCD
    plain = [xcd_strip_tile(w, n_rt, nstrip, False) for w in range(n_rt * nstrip)]
    assert plain == [(w % n_rt, w // n_rt) for w in range(n_rt * nstrip)]   # row tile fastest


def gemm_tile(wg, n_pt, n_rt, per_xcd, band=4):
    """The two-body split-BF16 GEMM's (column tile P, column tile R) of
    workgroup wg (k_gemm_tn_lds): XCD wg % 8 takes the contiguous range
    [xcd per_xcd, (xcd + 1) per_xcd) of a banded order (bands of `band` P
    tiles, R fastest within a band); ids past the tiles return None."""
    loc, t = wg >> 3, (wg & 7) * per_xcd + (wg >> 3)
    if loc >= per_xcd or t >= n_pt * n_rt:
        return None
    b = min(t // (band * n_rt), (n_pt - 1) // band)
    r = t - b * band * n_rt
    gw = min(band, n_pt - b * band)
    return b * band + r % gw, r // gw


@pytest.mark.parametrize("n_pt,n_rt", [(33, 33), (1, 1), (5, 3), (4, 9), (9, 4), (17, 2), (2, 17)])
def test_gemm_tile_map_is_a_bijection_and_xcd_ranges_are_compact(n_pt, n_rt):
    per = (n_pt * n_rt + 7) // 8
    tiles = [gemm_tile(w, n_pt, n_rt, per) for w in range(8 * per)]
    got = [t for t in tiles if t is not None]
    assert len(got) == n_pt * n_rt and set(got) == {(p, r) for p in range(n_pt) for r in range(n_rt)}
    # the first 32 tiles an XCD runs (its resident set) span few P and R tiles
    for x in range(8):
        first = [tiles[8 * loc + x] for loc in range(min(per, 32)) if tiles[8 * loc + x] is not None]
        if len(first) >= 32:
            assert len({p for p, _ in first}) <= 8 and len({r for _, r in first}) <= 9
