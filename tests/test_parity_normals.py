"""GPU parity of the PCA step of the normals (Section 3.4 "Approach
directions"): the library's device routine (through af_pca_axes) against the
oracle's on the same neighbourhood moments, bit for bit.  The moments cover
random neighbourhoods of every size the kNN can produce, tight spectra,
collinear and planar sets, and the degenerate counts below 3.  Both sides run
cyclic Jacobi with IEEE basic operations only, so any difference in the GPU's
division or square-root rounding shows up here."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

WIN = np.array([(x, y, z) for z in range(-3, 4) for y in range(-3, 4) for x in range(-3, 4)])


def moment_rows(sets):
    rows = np.zeros((len(sets), 10), np.int32)
    for i, d in enumerate(sets):
        d = np.asarray(d, np.int64).reshape(-1, 3)
        rows[i, 0] = len(d)
        if len(d):
            rows[i, 1:4] = d.sum(0)
            rows[i, 4:] = [(d[:, a] * d[:, b]).sum()
                           for a, b in ((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))]
    return rows


def test_pca_axes_bit_exact(oracle_mod):
    from paper_2608_06412_amd.af import pca_axes
    rng = np.random.default_rng(123)
    sets = []
    for it in range(60000):
        k = int(rng.integers(0, 30))
        sets.append(WIN[rng.choice(len(WIN), size=k, replace=False)])
    # collinear, planar, whole window, symmetric shells
    for ax in range(3):
        line = np.zeros((7, 3), np.int64)
        line[:, ax] = np.arange(-3, 4)
        sets.append(line)
        sets.append(WIN[WIN[:, ax] == 0])
    sets.append(WIN)
    for d2 in range(1, 28):
        sh = WIN[(WIN ** 2).sum(1) == d2]
        if len(sh):
            sets.append(sh)
    rows = moment_rows(sets)
    print("%d neighbourhoods" % len(rows), flush=True)
    ga, gh = pca_axes(rows)
    oa, oh = oracle_mod.pca_axes(rows)
    assert np.array_equal(gh, oh)
    bad = np.nonzero(np.any(ga != oa, axis=1))[0]
    assert len(bad) == 0, (len(bad), rows[bad[:5]], ga[bad[:5]], oa[bad[:5]])
    assert int(gh.sum()) > 50000
