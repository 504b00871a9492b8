"""Pins of the oracle's channels-and-inclusions coefficient (the high-contrast
synthetic medium standing in for the figure-only media of Secs. 5.1-5.2)."""
import numpy as np

from oracle import core
from paper_1607_00693_amd import workloads as W


def _theta(x, decades=4.0):
    return 10.0 ** (decades / (1.0 + np.exp(-x)))


def test_single_features_cover_hand_counted_cells():
    nf = 10
    # horizontal channel at y = 0.3 from x = 0.2 to 0.7: row 3, centroids
    # 0.25 .. 0.65 -> columns 2..6
    a = core.coef_features(np.array([[0.7]]), nf, [0], [0.2], [0.3], [0.5])[0]
    want = np.ones((nf, nf))
    want[3, 2:7] = _theta(0.7)
    np.testing.assert_allclose(a, want, rtol=1e-15)
    # vertical channel at x = 0.95 from y = 0.52 (clipped at the top): column
    # 9, rows 5..9 (centroids 0.55 .. 0.95 <= 0.52 + 0.6)
    a = core.coef_features(np.array([[-1.3]]), nf, [1], [0.95], [0.52], [0.6])[0]
    want = np.ones((nf, nf))
    want[5:10, 9] = _theta(-1.3)
    np.testing.assert_allclose(a, want, rtol=1e-15)
    # square of side 0.2 centred at (0.5, 0.5): centroids 0.45, 0.55 in each
    # direction -> 2 x 2 cells
    a = core.coef_features(np.array([[2.0]]), nf, [2], [0.5], [0.5], [0.2])[0]
    want = np.ones((nf, nf))
    want[4:6, 4:6] = _theta(2.0)
    np.testing.assert_allclose(a, want, rtol=1e-15)


def test_later_feature_overrides_and_contrast_limits():
    nf = 8
    kind, x0, y0, size = [0, 2], [0.0, 0.5], [0.5, 0.5], [1.0, 0.25]
    xi = np.array([[0.0, 40.0], [-40.0, 0.0]])
    a = core.coef_features(xi, nf, kind, x0, y0, size)
    # row 4 is the channel; the square covers rows/cols 3..4 and wins on (4, 3..4)
    assert np.allclose(a[0, 4, [0, 1, 2, 5, 6, 7]], 100.0)           # sigmoid(0) = 1/2 -> 10^2
    np.testing.assert_allclose(a[0, 3:5, 3:5], 1e4, rtol=1e-12)      # sigmoid(40) ~ 1
    np.testing.assert_allclose(a[1, 4, [0, 7]], 1.0, rtol=1e-12)     # sigmoid(-40) ~ 0
    np.testing.assert_allclose(a[1, 3:5, 3:5], 100.0, rtol=1e-15)
    assert (a[:, :3] == 1.0).all() and (a[:, 5:] == 1.0).all()


def test_workload_medium_contrast_and_coverage():
    wl = W.CHANNELS64
    kind, x0, y0, size = W.channel_geometry(wl)
    assert (kind[:wl.nchan] <= 1).all() and (kind[wl.nchan:] == 2).all()
    nf = 8 * wl.nc
    xi = np.zeros((1, wl.nxi))
    a = core.coef_features(xi, nf, kind, x0, y0, size)[0]
    assert set(np.unique(a)) == {1.0, 100.0}
    # a channel that nothing later crosses covers about length * nf cells of
    # its row or column
    covered = (a == 100.0).mean()
    assert 0.01 < covered < 0.1
