"""Seeded synthetic inputs shared by the GPU path, the oracle and the tests.

This module only draws random numbers and records workload sizes: it holds
none of the method's arithmetic (no coefficient formula, no assembly, no
solve).  The random variables xi are drawn on the host with numpy's PCG64
(``numpy.random.default_rng(seed)``) and handed to both sides.

Workloads (synthetic stand-ins: the paper's own media exist only as figures):

* ``mesh8``   -- 8 x 8 coarse elements, H/h = 8 (64 x 64 fine Q1), 16 bumps of
  radius 1/4 on a 4 x 4 grid, oscillation period eps = 1/32, xi ~ U[-1,1]^16.
* ``mesh32``  -- 32 x 32 coarse elements, H/h = 32 (1024 x 1024 fine Q1), 64
  bumps of radius 1/8 on an 8 x 8 grid, eps = 1/256, xi ~ U[-1,1]^64,
  4096 samples.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass(frozen=True)
class BumpWorkload:
    name: str
    nc: int          # coarse elements per direction
    m: int           # fine cells per coarse element per direction (H/h)
    nsamples: int
    g: int           # bumps per direction (g*g random variables)
    rho: float       # bump radius
    eps: float       # oscillation period
    seed: int
    base: float = 2.0
    amp: float = 1.8
    beta: float = 0.5

    @property
    def nfine(self) -> int:
        return self.nc * self.m

    @property
    def nxi(self) -> int:
        return self.g * self.g

    @property
    def M(self) -> int:
        return self.nc * self.nc

    def coef_params(self) -> dict:
        return dict(g=self.g, rho=self.rho, eps=self.eps, base=self.base, amp=self.amp, beta=self.beta)


MESH8 = BumpWorkload("mesh8_plain_fp64", nc=8, m=8, nsamples=64, g=4, rho=0.25, eps=1.0 / 32, seed=1001)
MESH32 = BumpWorkload("mesh32_plain", nc=32, m=32, nsamples=4096, g=8, rho=0.125, eps=1.0 / 256, seed=1002)


def uniform_xi(nsamples: int, nxi: int, seed: int) -> np.ndarray:
    """xi ~ U[-1,1]^nxi, i.i.d., shape [nsamples][nxi], float64."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=(nsamples, nxi))


def normal_xi(nsamples: int, nxi: int, seed: int) -> np.ndarray:
    """xi ~ N(0,1)^nxi, i.i.d., shape [nsamples][nxi], float64."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(size=(nsamples, nxi))


def uniform_array(shape, lo: float, hi: float, seed: int) -> np.ndarray:
    """Generic seeded uniform array (test coefficients, random SPD data)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=shape)


def lognormal_field(shape, sigma: float, seed: int) -> np.ndarray:
    """Element-wise independent log-normal coefficient exp(sigma * N(0,1))."""
    rng = np.random.default_rng(seed)
    return np.exp(sigma * rng.standard_normal(size=shape))


def permutation(n: int, seed: int) -> np.ndarray:
    """Seeded permutation of range(n) (minibatch order), int64."""
    return np.random.default_rng(seed).permutation(n).astype(np.int64)


def mlp_init(npatch: int, seed: int, kin: int = 4, width: int = 64, nout: int = 20) -> np.ndarray:
    """Initial surrogate weights [npatch][nparams] (float32): Glorot-uniform
    weights, zero biases, in the packing W1, b1, W2, b2, W3, b3, W4, b4."""
    rng = np.random.default_rng(seed)
    shapes = [(kin, width), (width,), (width, width), (width,), (width, width), (width,), (width, nout), (nout,)]
    parts = []
    for shp in shapes:
        if len(shp) == 2:
            lim = np.sqrt(6.0 / (shp[0] + shp[1]))
            parts.append(rng.uniform(-lim, lim, size=(npatch,) + shp).reshape(npatch, -1))
        else:
            parts.append(np.zeros((npatch, shp[0])))
    return np.concatenate(parts, axis=1).astype(np.float32)
