"""Element loads of the coarse system for a bilinear source (test
infrastructure only, see package doc).

The load of coarse element K and its local node l is b^K_l = int_K b p^l
(the Petrov-Galerkin load of eq. stiffness_local_petrov with the coarse
bilinear test functions p^l; with b = 1 every entry is H^2/4).  Sec. 5.3
takes the source b(x1, x2) = 2 + x1 x2; here b is any bilinear polynomial

    b(x, y) = f00 + f10 x + f01 y + f11 x y

on square coarse elements of side H = 1/ncx, element (kx, ky) =
[kx H, (kx+1) H] x [ky H, (ky+1) H], local nodes counter-clockwise from the
lower-left corner: p^0 = (1-s)(1-t), p^1 = s(1-t), p^2 = s t, p^3 = (1-s) t
with s = (x - x0)/H, t = (y - y0)/H.

Both b and p^l are products of a function of x and a function of y, so each
entry is a sum of products of one-dimensional integrals, written out here in
closed form: with x = x0 + H s,
    int (1-s) dx = H/2,         int s dx = H/2,
    int x (1-s) dx = H (x0/2 + H/6),   int x s dx = H (x0/2 + H/3).
"""
from __future__ import annotations

import numpy as np


def _moments(x0: float, H: float):
    """(int X dx, int x X dx) for X = 1 - s and X = s on [x0, x0 + H]."""
    return ((H / 2.0, H * (x0 / 2.0 + H / 6.0)),   # X = 1 - s
            (H / 2.0, H * (x0 / 2.0 + H / 3.0)))   # X = s


def element_loads_bilinear(ncx: int, ncy: int, f) -> np.ndarray:
    """b^K_l for every element: [ncy*ncx][4], element index ky*ncx + kx."""
    f00, f10, f01, f11 = (float(v) for v in f)
    H = 1.0 / ncx
    # local node l -> (x factor, y factor): 0 = (1-s, 1-t), 1 = (s, 1-t),
    # 2 = (s, t), 3 = (1-s, t); index 0 means "1 - s", 1 means "s"
    fac = [(0, 0), (1, 0), (1, 1), (0, 1)]
    out = np.zeros((ncy * ncx, 4))
    for ky in range(ncy):
        my = _moments(ky * H, H)
        for kx in range(ncx):
            mx = _moments(kx * H, H)
            for l, (ix, iy) in enumerate(fac):
                X0, X1 = mx[ix]  # int X, int x X
                Y0, Y1 = my[iy]
                out[ky * ncx + kx, l] = f00 * X0 * Y0 + f10 * X1 * Y0 + f01 * X0 * Y1 + f11 * X1 * Y1
    return out
