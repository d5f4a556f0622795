"""GPU test of nrto_project_soc_noalloc (the validated projection that
allocates nothing) through the C ABI: its output equals that of
nrto_project_soc with validation on two calls in a row, the second with a
smaller input, and it rejects offsets that nrto_project_soc rejects."""
import numpy as np
import pytest

import synth
from oracle import soc

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _case(seed, n, hi):
    L = synth.cone_lengths(seed, n, 1, hi)
    L[::5] = 0
    off = np.concatenate([[0], np.cumsum(L)]).astype(np.int64)
    x = 2.0 * synth.cone_values(seed + 1, int(off[-1]))
    return x, off


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_noalloc_matches_allocating_entry_point_twice(dtype):
    torch = _torch()
    from paper_2603_02642_amd import nrto
    tdt = torch.float64 if dtype == "f64" else torch.float32
    for seed, n, hi in ((11, 4000, 2000), (13, 300, 100)):   # second call smaller
        x, off = _case(seed, n, hi)
        xd = torch.from_numpy(x).to(device="cuda", dtype=tdt)
        od = torch.from_numpy(off).cuda()
        print(f"noalloc case dtype={dtype} seed={seed} cones={n} entries={off[-1]}", flush=True)
        ref = nrto.project_soc(xd, od, validate=True)
        got = nrto.project_soc_noalloc(xd, od)
        torch.cuda.synchronize()
        assert torch.equal(got, ref)
        exact = soc.project_segments(xd.double().cpu().numpy(), off)
        tol = 1e-12 if dtype == "f64" else 1e-5
        err = np.max(np.abs(got.double().cpu().numpy() - exact) / np.maximum(1.0, np.abs(exact)))
        assert err <= tol, err


def test_noalloc_rejects_bad_offsets_then_recovers():
    torch = _torch()
    from paper_2603_02642_amd import nrto
    x, off = _case(17, 500, 64)
    xd = torch.from_numpy(x).cuda()
    bad = off.copy()
    bad[10], bad[11] = bad[11], bad[10] - 1          # decreasing pair, ends still valid
    with pytest.raises(nrto.NrtoError):
        nrto.project_soc_noalloc(xd, torch.from_numpy(bad).cuda())
    with pytest.raises(nrto.NrtoError):
        nrto.project_soc(xd, torch.from_numpy(bad).cuda(), validate=True)
    # the flag left set by the rejected call is cleared by the next call
    od = torch.from_numpy(off).cuda()
    got = nrto.project_soc_noalloc(xd, od)
    ref = nrto.project_soc(xd, od, validate=True)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
