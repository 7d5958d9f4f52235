"""The FP32 kernels' shortcut for the re-emission bin (reading R8) against the
plain draw.

Plain draw (oracle, FP64 kernels): a* uniform in the slice [a_lo, a_hi] of
absorbed power per mass, bin = number of G-table points <= a*.  Shortcut (FP32
kernels): bin = number of points <= a_lo; only when the first point above a_lo
lies inside the slice is a* drawn and the bin searched again.  Both must give
the same bin for every uniform, so the two layouts differ only in which Philox
words feed the other draws, which are independent uniforms either way.
"""
import numpy as np


def count_le(G, x):
    return int(np.searchsorted(G, x, side="right"))


def plain_bin(G, lo, hi, u):
    return count_le(G, lo + u * (hi - lo))


def shortcut_bin(G, lo, hi, u):
    row = count_le(G, lo)
    if row < len(G) and G[row] <= hi:
        row = count_le(G, lo + u * (hi - lo))
    return row


def test_shortcut_equals_plain_draw_for_every_uniform():
    rng = np.random.default_rng(7)
    G = np.sort(rng.lognormal(0.0, 3.0, 512))
    n_straddle = 0
    for _ in range(4000):
        lo = float(np.exp(rng.uniform(np.log(G[0]) - 1, np.log(G[-1]) + 1)))
        # slices from tiny (inside one bin) to wide (over several bin edges)
        hi = lo * (1 + 10 ** rng.uniform(-7, 0.5))
        straddle = count_le(G, lo) < len(G) and G[count_le(G, lo)] <= hi
        n_straddle += straddle
        for u in (0.0, 1.0 - 2**-33, *rng.random(8)):
            assert shortcut_bin(G, lo, hi, u) == plain_bin(G, lo, hi, u)
    # both kinds of slices were exercised
    assert 200 < n_straddle < 3800


def test_slice_on_a_table_point():
    # a slice whose upper end is a table point straddles it (the point is <= a_hi)
    G = np.array([1.0, 2.0, 4.0, 8.0])
    for u in (0.0, 0.5, 1.0):
        assert shortcut_bin(G, 1.5, 2.0, u) == plain_bin(G, 1.5, 2.0, u)
    # below and above the table
    assert shortcut_bin(G, 0.1, 0.2, 0.3) == plain_bin(G, 0.1, 0.2, 0.3) == 0
    assert shortcut_bin(G, 9.0, 9.5, 0.3) == plain_bin(G, 9.0, 9.5, 0.3) == 4
