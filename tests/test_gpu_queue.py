"""One persistent launch over batches of several H/h (m = 8, 16, 32) through
the C-ABI (stomsfem_upscale_queue).

Every pair runs the same device code as the per-m kernels, so S and the
per-pair status must equal stomsfem_upscale's bit for bit; one small mixed
set is also checked against the CPU oracle at the plain path's tolerance
(per pair, max_q |S_q - S_q^ref| <= 1e-10 max_q |S_q^ref|).  Pair counts are
ragged against the work items (6 pairs for m = 16, 32; 64 for m = 8).
"""
import ctypes
import sys

import numpy as np
import pytest
import torch

from paper_1607_00693_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-queue] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sm():
    from paper_1607_00693_amd import stomsfem

    assert torch.cuda.is_available()
    stomsfem.lib()
    return stomsfem


def _batches(sm, specs, seed, dtype=np.float64):
    """specs: (m, ncx, ncy, N) -> list of (a_np, a, S, status, batch)."""
    out = []
    for i, (m, ncx, ncy, N) in enumerate(specs):
        a_np = W.lognormal_field((N, ncy * m, ncx * m), 1.0, seed + 17 * i).astype(dtype)
        a = torch.from_numpy(a_np).cuda()
        S = torch.full((N, ncx * ncy, 10), np.nan, dtype=torch.float64, device="cuda")
        st = torch.full((N, ncx * ncy), 99, dtype=torch.int32, device="cuda")
        out.append((a_np, a, S, st, sm.make_batch(a, ncx, ncy, m, S, st)))
    return out


def _per_batch(sm, specs, bs):
    ref = []
    for (m, ncx, ncy, N), (_, a, _, _, _) in zip(specs, bs):
        st = torch.full((N, ncx * ncy), 99, dtype=torch.int32, device="cuda")
        ref.append((sm.upscale(a, ncx, ncy, m, status=st), st))
    return ref


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_mixed_batches_bitwise_equal_to_per_m_kernels(sm, dtype):
    # batches listed out of cost order; pair counts 7*5*3=105 (m=8: one full
    # item of 64 and a ragged one), 3*2*5=30, 3*2*3=18 (m=32: three items, an
    # odd count, so that some workgroup holds an m = 32 and an m = 16 item at
    # once), plus a second m = 8 batch
    specs = [(8, 7, 5, 3), (32, 3, 2, 3), (16, 3, 2, 5), (8, 3, 3, 1)]
    say(f"mixed batches {specs} dtype={np.dtype(dtype).name}")
    bs = _batches(sm, specs, 4100, dtype)
    sm.upscale_queue([b[4] for b in bs])
    ref = _per_batch(sm, specs, bs)
    torch.cuda.synchronize()
    for (spec, b, (S_ref, st_ref)) in zip(specs, bs, ref):
        assert torch.equal(b[2], S_ref), spec
        assert torch.equal(b[3], st_ref), spec
        assert (b[3] == sm.OK).all()


def test_mixed_batches_match_oracle(sm, orc):
    specs = [(16, 2, 3, 2), (8, 3, 2, 2), (32, 2, 1, 2)]
    say(f"mixed batches against the oracle {specs}")
    bs = _batches(sm, specs, 4200)
    sm.upscale_queue([b[4] for b in bs])
    torch.cuda.synchronize()
    for (m, ncx, ncy, N), b in zip(specs, bs):
        S_ref, _, _ = orc.upscale(b[0], ncx, ncy, m)
        S = b[2].cpu().numpy()
        err = (np.abs(S - S_ref).max(-1) / np.abs(S_ref).max(-1)).max()
        say(f"m={m}: max rel err {err:.2e}")
        assert err < 1e-10


def test_repeated_calls_and_bad_pivots(sm):
    # the item counter is reset by every call; a non-positive coefficient
    # flags only its own pair, as in the per-m kernels
    specs = [(32, 2, 2, 1), (8, 2, 2, 3), (16, 2, 2, 2)]
    say("repeated calls, bad pivots")
    bs = _batches(sm, specs, 4300)
    bs[1][1][1, 3, 12] = -50.0   # m = 8: sample 1, element (1, 0)
    bs[2][1][0, 20, 5] = np.nan  # m = 16: sample 0, element (0, 1)
    for _ in range(3):
        sm.upscale_queue([b[4] for b in bs])
    ref = _per_batch(sm, specs, bs)
    torch.cuda.synchronize()
    for (spec, b, (S_ref, st_ref)) in zip(specs, bs, ref):
        ok = (st_ref == sm.OK)
        assert torch.equal(b[2][ok], S_ref[ok]), spec
        assert torch.equal(b[3], st_ref), spec
    assert int(bs[1][3][1, 1]) == sm.ENOTSPD and int((bs[1][3] != sm.OK).sum()) == 1
    assert int(bs[2][3][0, 2]) == sm.ENOTSPD and int((bs[2][3] != sm.OK).sum()) == 1


def test_empty_and_invalid_arguments(sm):
    say("empty and invalid arguments")
    # an empty batch beside a real one
    bs = _batches(sm, [(8, 2, 2, 0), (16, 2, 2, 1)], 4400)
    sm.upscale_queue([b[4] for b in bs])
    torch.cuda.synchronize()
    assert (bs[1][3] == sm.OK).all() and torch.isfinite(bs[1][2]).all()
    # m outside {8, 16, 32}
    bad = _batches(sm, [(12, 2, 2, 1)], 4500)
    with pytest.raises(sm.StomsfemError) as e:
        sm.upscale_queue([bad[0][4]])
    assert e.value.code == sm.EINVAL
    # mixed coefficient types
    b64 = _batches(sm, [(8, 2, 2, 1)], 4600)
    b32 = _batches(sm, [(16, 2, 2, 1)], 4700, np.float32)
    with pytest.raises(sm.StomsfemError) as e:
        sm.upscale_queue([b64[0][4], b32[0][4]])
    assert e.value.code == sm.EINVAL
    # more than eight batches, or none
    many = _batches(sm, [(8, 2, 2, 1)] * 9, 4800)
    with pytest.raises(sm.StomsfemError) as e:
        sm.upscale_queue([b[4] for b in many])
    assert e.value.code == sm.EINVAL
    rc = sm.lib().stomsfem_upscale_queue(None, 0, None)
    assert rc == sm.EINVAL
    # host memory is rejected before anything is queued
    a_host = torch.ones((1, 16, 16), dtype=torch.float64)
    S_dev = torch.empty((1, 4, 10), dtype=torch.float64, device="cuda")
    b = sm.Batch(2, 2, 8, sm.F64, 1, a_host.data_ptr(), S_dev.data_ptr(), None)
    rc = sm.lib().stomsfem_upscale_queue(ctypes.byref(b), 1, None)
    assert rc == sm.EINVAL


def test_graph_capture_replays(sm):
    # the launch (counter reset kernel + persistent kernel) captured in a HIP
    # graph: every replay, with eager work and synchronisation between the
    # replays, equals the eager result bit for bit
    specs = [(16, 3, 3, 2), (32, 2, 2, 1), (8, 4, 4, 2)]
    say("graph capture")
    bs = _batches(sm, specs, 4900)
    batches = [b[4] for b in bs]
    sm.upscale_queue(batches)  # eager run (also sets up the library workspace)
    torch.cuda.synchronize()
    eager = [(b[2].clone(), b[3].clone()) for b in bs]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        sm.upscale_queue(batches, stream=s)
    torch.cuda.synchronize()
    for rep in range(3):
        for b in bs:
            b[2].fill_(float("nan"))
            b[3].fill_(99)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for (spec, b, (S_e, st_e)) in zip(specs, bs, eager):
            assert torch.equal(b[2], S_e), (rep, spec)
            assert torch.equal(b[3], st_e), (rep, spec)
    del g
