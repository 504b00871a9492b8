"""Pins of the oracle's element loads for a bilinear source (Sec. 5.3 takes
b = 2 + x1 x2; the load is int_K b p^l, reading 5): the constant source's
closed form H^2/4, the partition of unity (the four loads of an element sum
to int_K b, which the midpoint rule gives exactly for a bilinear b), brute
force quadrature of b p^l, and the x <-> y mirror symmetry of 2 + x y."""
import numpy as np
import pytest
from scipy import integrate

from oracle import loads


def test_constant_source_is_quarter_element_area():
    for ncx, ncy in ((1, 1), (4, 4), (5, 3)):
        b = loads.element_loads_bilinear(ncx, ncy, (1.0, 0.0, 0.0, 0.0))
        assert np.allclose(b, 0.25 / ncx**2, rtol=1e-15, atol=0)


@pytest.mark.parametrize("f", [(2.0, 0.0, 0.0, 1.0), (0.3, -1.2, 0.7, 2.5)])
def test_loads_sum_to_element_integral(f):
    ncx, ncy = 6, 4
    H = 1.0 / ncx
    b = loads.element_loads_bilinear(ncx, ncy, f)
    for ky in range(ncy):
        for kx in range(ncx):
            xc, yc = (kx + 0.5) * H, (ky + 0.5) * H
            whole = H * H * (f[0] + f[1] * xc + f[2] * yc + f[3] * xc * yc)
            assert abs(b[ky * ncx + kx].sum() - whole) <= 1e-15 * max(1.0, abs(whole))


def test_brute_force_quadrature():
    f = (2.0, 0.4, -0.3, 1.0)
    ncx, ncy = 3, 2
    H = 1.0 / ncx
    b = loads.element_loads_bilinear(ncx, ncy, f)
    src = lambda x, y: f[0] + f[1] * x + f[2] * y + f[3] * x * y  # noqa: E731
    for (kx, ky) in ((0, 0), (2, 1), (1, 1)):
        x0, y0 = kx * H, ky * H
        p = [lambda x, y: (1 - (x - x0) / H) * (1 - (y - y0) / H), lambda x, y: ((x - x0) / H) * (1 - (y - y0) / H),
             lambda x, y: ((x - x0) / H) * ((y - y0) / H), lambda x, y: (1 - (x - x0) / H) * ((y - y0) / H)]
        for l in range(4):
            ref, _ = integrate.dblquad(lambda y, x: src(x, y) * p[l](x, y), x0, x0 + H, y0, y0 + H,
                                       epsabs=1e-15, epsrel=1e-13)
            assert abs(b[ky * ncx + kx, l] - ref) <= 1e-12 * abs(ref)


def test_mirror_symmetry_of_the_paper_source():
    n = 5
    b = loads.element_loads_bilinear(n, n, (2.0, 0.0, 0.0, 1.0))
    swap = [0, 3, 2, 1]  # x <-> y exchanges local nodes 1 and 3
    for ky in range(n):
        for kx in range(n):
            np.testing.assert_allclose(b[kx * n + ky][swap], b[ky * n + kx], rtol=1e-15, atol=0)
