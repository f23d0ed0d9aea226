"""The allocation-free re-distancing entry point (mpp_ls_reinit_noalloc) against the
entry point it varies (mpp_ls_reinit with a caller-owned work array): bit for bit, on two
calls in a row of which the second is smaller (the library's scratch field keeps the first
call's contents), with odd and even step counts (the result ends in the scratch field or
in phi), and at the largest size the scratch field takes.  Collected last on purpose."""
import ctypes

import numpy as np
import pytest

import oracle as O
from paper_2312_11740_amd import problems as G

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2312_11740_amd as M  # noqa: E402

DEV = "cuda:0"


def noisy_phi(n, batch, seed):
    rng = np.random.default_rng(seed)
    out = []
    for b in range(batch):
        c = rng.uniform(0.35, 0.65, 3)
        ph = G.bubble_phi(n, [tuple(c)], [0.2 + 0.05 * b])
        out.append(ph * rng.uniform(0.5, 2.5) + 0.1 * ph ** 2)   # not a distance
    return np.stack(out) if batch > 1 else out[0]


def run_both(n, batch, iters, seed):
    ph = noisy_phi(n, batch, seed)
    phi0 = torch.from_numpy(ph).to(DEV)
    ref = M.ls_reinit(phi0.clone(), iters, phi0=phi0)            # mpp_ls_reinit + work array
    phi = phi0.clone()
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    st = M.load_library().mpp_ls_reinit_noalloc(
        n, batch, ctypes.c_void_p(phi0.data_ptr()), ctypes.c_void_p(phi.data_ptr()), iters,
        0.5 / n, M._stream_handle(phi.device))
    torch.cuda.synchronize()
    assert st == M.OK
    assert torch.cuda.memory_allocated() == before
    print("noalloc reinit n=%d batch=%d iters=%d" % (n, batch, iters), flush=True)
    return ph, ref, phi


def test_noalloc_reinit_two_calls_second_smaller():
    ph, ref, got = run_both(64, 2, 3, 1)
    assert torch.equal(got, ref)
    assert not torch.equal(got, torch.from_numpy(ph).to(DEV))
    ph2, ref2, got2 = run_both(40, 1, 4, 2)
    assert torch.equal(got2, ref2)
    # and the second against the oracle (the existing entry point's own bar)
    assert np.array_equal(got2.cpu().numpy(), O.ls_reinit(ph2, ph2, 4, 0.5 / 40))


def test_noalloc_reinit_at_the_largest_size():
    ph, ref, got = run_both(256, 1, 1, 3)
    assert torch.equal(got, ref)


def test_noalloc_reinit_refuses_more_than_its_scratch():
    phi = torch.zeros((2, 256, 256, 256), dtype=torch.float64, device=DEV)
    with pytest.raises(M.MppError) as ei:
        M.ls_reinit_noalloc(phi, phi.clone(), 2)
    assert ei.value.status == M.ENOMEM
