"""The allocation-free orbital gradient (hci_orbital_gradient_noalloc) against
hci_orbital_gradient, through the C ABI: two calls in a row on one GPU, the
second with a smaller orbital count (so a smaller share of the fixed scratch
array that both calls reuse), and each result equal to the allocating entry
point's bit for bit (the same kernels with the same split; the bar of the
orbital step's parity tests, 1e-12 of the largest entry, is implied).  The
calls allocate nothing through the context's allocator.
"""
import numpy as np
import pytest
import torch

import hci_synth as hs

pytestmark = pytest.mark.gpu


def _sym_tensors(n, seed):
    rng = np.random.default_rng(seed)
    r1 = rng.normal(size=(n, n))
    r1 = r1 + r1.T
    r2 = rng.normal(size=(n, n, n, n))
    r2 = r2 + r2.transpose(2, 3, 0, 1)
    r2 = r2 + r2.transpose(1, 0, 3, 2)
    return r1, r2


def test_noalloc_gradient_matches_allocating_entry_point(gpu_available):
    import paper_1708_07544_amd as P
    from paper_1708_07544_amd import _lib

    dev = torch.device("cuda:0")
    for n, seed in ((44, 11), (16, 12)):
        print(f"no-alloc gradient: n={n} seed={seed}", flush=True)
        h, g = hs.make_integrals(n, 3 * n, seed)
        ctx = P.HCIContext(h, g, n // 2, n // 2)
        r1, r2 = _sym_tensors(n, seed)
        t1 = torch.tensor(r1, dtype=torch.float64, device=dev)
        t2 = torch.tensor(r2, dtype=torch.float64, device=dev)
        ref = ctx.orbital_gradient(t1, t2)
        got = torch.full((n, n), float("nan"), dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated(dev)
        rc = _lib.lib().hci_orbital_gradient_noalloc(ctx.handle, _lib._ptr(t1), _lib._ptr(t2), _lib._ptr(got),
                                                      _lib._stream())
        assert rc == _lib.HCI_OK, _lib.lib().hci_last_error()
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated(dev) == before
        a, b = got.cpu().numpy(), ref.cpu().numpy()
        assert np.isfinite(a).all()
        assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()
        assert np.array_equal(a, b)
        # the binding method gives the same
        got2 = torch.zeros((n, n), dtype=torch.float64, device=dev)
        ctx.orbital_gradient_noalloc(t1, t2, got2)
        assert torch.equal(got2, ref)


def test_noalloc_gradient_rejects_bad_arguments(gpu_available):
    import paper_1708_07544_amd as P
    from paper_1708_07544_amd import _lib

    n = 6
    h, g = hs.make_integrals(n, 18, 3)
    ctx = P.HCIContext(h, g, 3, 3)
    rc = _lib.lib().hci_orbital_gradient_noalloc(ctx.handle, None, None, None, _lib._stream())
    assert rc == _lib.HCI_E_ARG
    assert _lib.lib().hci_orbital_gradient_noalloc(None, None, None, None, None) == _lib.HCI_E_ARG
    assert b"null" in _lib.lib().hci_last_error()
