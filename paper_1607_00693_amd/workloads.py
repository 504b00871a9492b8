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
* ``channels64`` -- 64 x 64 coarse elements, 8192 samples in 32 batches of
  256, H/h drawn per batch from {8, 16, 32}; background 1 plus 40 thin
  channels and 40 square inclusions (80 variables, xi ~ N(0,1)^80), each
  feature's conductivity set by its variable with up to four decades of
  contrast.
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


@dataclasses.dataclass(frozen=True)
class ChannelWorkload:
    name: str = "channels64"
    nc: int = 64
    nbatch: int = 32
    batch: int = 256          # samples per batch
    m_choices: tuple = (8, 16, 32)
    nchan: int = 40
    nsq: int = 40
    decades: float = 4.0      # conductivity 10^(decades * sigmoid(xi_j))
    geom_seed: int = 3005
    m_seed: int = 4005
    xi_seed: int = 1005

    @property
    def nxi(self) -> int:
        return self.nchan + self.nsq

    @property
    def M(self) -> int:
        return self.nc * self.nc


CHANNELS64 = ChannelWorkload()


def channel_geometry(wl: ChannelWorkload = CHANNELS64):
    """Feature geometry in continuous coordinates of the unit square:
    (kind int32 [nf], x0, y0, size float64 [nf]).  Channels 0..nchan-1: kind
    0 (horizontal) or 1 (vertical) with probability 1/2, start point
    (x0, y0) ~ U[0,1]^2, length ~ U[0.25, 1].  Squares: kind 2, centre
    (x0, y0) ~ U[0,1]^2, side ~ U[1/256, 1/64]."""
    rng = np.random.default_rng(wl.geom_seed)
    orient = rng.integers(0, 2, size=wl.nchan)
    start = rng.uniform(0.0, 1.0, size=(wl.nchan, 2))
    length = rng.uniform(0.25, 1.0, size=wl.nchan)
    centre = rng.uniform(0.0, 1.0, size=(wl.nsq, 2))
    side = rng.uniform(1.0 / 256, 1.0 / 64, size=wl.nsq)
    kind = np.concatenate([orient, np.full(wl.nsq, 2)]).astype(np.int32)
    x0 = np.concatenate([start[:, 0], centre[:, 0]])
    y0 = np.concatenate([start[:, 1], centre[:, 1]])
    size = np.concatenate([length, side])
    return kind, x0, y0, size


def batch_m(wl: ChannelWorkload = CHANNELS64) -> np.ndarray:
    """H/h of each batch, drawn uniformly from wl.m_choices."""
    rng = np.random.default_rng(wl.m_seed)
    return np.asarray(wl.m_choices)[rng.integers(0, len(wl.m_choices), size=wl.nbatch)].astype(np.int32)


@dataclasses.dataclass(frozen=True)
class GaussWorkload:
    """Stand-in for the short-correlation Gaussian medium of Sec. 5.3:
    kappa = 0.1 + exp(beta), beta a centred Gaussian field with covariance
    exp(-dx^2/l1^2 - dy^2/l2^2), sampled by the randomized spectral method
    with nterms cosines; coarse elements of H = 1/nc span H/l2 = 2
    correlation lengths in y (the paper's oversampled patch of 2H with
    l2 = H: two lengths; four local KL terms then hold >= 99%)."""
    name: str = "gauss16"
    nc: int = 16
    m: int = 16
    l1: float = 1.0
    l2: float = 1.0 / 32
    nterms: int = 256
    nsamples: int = 1024
    kl_terms: int = 4
    box: float = 3.0
    seed: int = 5005

    @property
    def nfine(self) -> int:
        return self.nc * self.m

    @property
    def M(self) -> int:
        return self.nc * self.nc


GAUSS16 = GaussWorkload()


def spectral_draws(nsamples: int, nterms: int, seed: int):
    """Random numbers of the spectral method: standard normals z
    [nsamples][nterms][2] (the wave vectors before scaling) and uniforms u
    [nsamples][nterms] on [0, 1) (the phases before scaling by 2 pi)."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal(size=(nsamples, nterms, 2))
    u = rng.uniform(0.0, 1.0, size=(nsamples, nterms))
    return z, u
