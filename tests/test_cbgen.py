"""The counter-based input generator (cbgen.c, CPU).

Pins: the Philox4x32-10 known-answer vectors published with the Random123
library (Salmon et al., SC 2011), the R-MAT quadrant rule on the first
draws, and the CSR build against numpy's stable sort."""

import numpy as np

from paper_2111_12493_amd import graphgen as gg


def test_philox_known_answers():
    assert gg.philox4x32_10([0, 0, 0, 0], [0, 0]) == (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)
    assert gg.philox4x32_10([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2) == (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)
    assert gg.philox4x32_10([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344], [0xA4093822, 0x299F31D0]) == \
        (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)


def _edges(scale, m, seed=27):
    L = gg._cbgen()
    src = np.empty(m, np.uint32)
    dst = np.empty(m, np.uint32)
    lab = np.empty(m, np.uint32)
    assert L.cb_rmat_edges(seed, scale, m, 0.57, 0.19, 0.19, 16, 1.2, src.ctypes.data, dst.ctypes.data,
                           lab.ctypes.data, 0) == 0
    return src, dst, lab


def test_rmat_quadrants_follow_the_draws():
    # edge i, level l: word l % 4 of Philox((i, 0, l // 4, 0), (seed, 0))
    scale, m = 9, 40
    src, dst, _ = _edges(scale, m)
    A, AB, ABC = (int(np.floor(x * 2 ** 32)) for x in (0.57, 0.76, 0.95))
    for i in range(m):
        s = d = 0
        for lvl in range(scale):
            u = gg.philox4x32_10([i, 0, lvl // 4, 0], [27, 0])[lvl % 4]
            s = 2 * s + (u >= AB)
            d = 2 * d + ((A <= u < AB) or u >= ABC)
        assert (int(src[i]), int(dst[i])) == (s, d), i


def test_csr_is_the_stable_sort_by_source():
    g = gg.cb_rmat_graph(14, 1 << 17, n_types=64, n_labels=16, seed=5)
    src, dst, lab = _edges(14, 1 << 17, seed=5)
    order = np.argsort(src, kind="stable")
    assert np.array_equal(g.tgt, dst[order])
    assert np.array_equal(np.diff(g.row_off.astype(np.int64)), np.bincount(src, minlength=g.n))
    assert g.lab.max() < 16 and g.typ.max() < 64
    counts = np.diff(g.typ_off.astype(np.int64))
    assert counts.min() >= 0 and counts.max() <= 4


def test_deterministic_and_labels_u16():
    a = gg.make_config("cb_rmat16")
    b = gg.make_config("cb_rmat16")
    assert a.lab.dtype == np.uint16
    for f in ("row_off", "tgt", "lab", "typ_off", "typ"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f
