"""Calls that share the library workspace, queued on two streams at once,
give the results of the same calls on one stream (the workspace users order
themselves with events), and calls on one model from two streams likewise.
Bit-for-bit comparisons: the kernels and their inputs are the same."""
import numpy as np
import pytest
import torch

from paper_1607_00693_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sm():
    from paper_1607_00693_amd import stomsfem

    stomsfem.lib()
    return stomsfem


def _S(sm, wl, N, seed):
    xi = torch.from_numpy(W.uniform_xi(N, wl.nxi, seed)).cuda()
    return sm.upscale(sm.coef_bumps(xi, wl.nfine, **wl.coef_params()), wl.nc, wl.nc, wl.m)


def test_coarse_solves_on_two_streams_match_one_stream(sm):
    print("[gpu-streams] coarse solves on two streams", flush=True)
    wl = W.MESH8
    S1, S2 = _S(sm, wl, 4096, 7301), _S(sm, wl, 4096, 7302)
    torch.cuda.synchronize()
    U1, m1, v1 = sm.coarse_solve(S1, wl.nc, wl.nc)
    U2, m2, v2 = sm.coarse_solve(S2, wl.nc, wl.nc)
    torch.cuda.synchronize()
    ref = [t.cpu().numpy() for t in (U1, m1, v1, U2, m2, v2)]
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    for _ in range(3):
        with torch.cuda.stream(sa):
            A = sm.coarse_solve(S1, wl.nc, wl.nc, stream=sa)
        with torch.cuda.stream(sb):
            B = sm.coarse_solve(S2, wl.nc, wl.nc, stream=sb)
        torch.cuda.synchronize()
        got = [t.cpu().numpy() for t in (*A, *B)]
        for g, r in zip(got, ref):
            np.testing.assert_array_equal(g, r)
