"""bl_gram_noalloc, the Gram product for callers that cannot allocate device memory, through
the C ABI against bl_gram (same kernels and summation order: bit-identical) and against a
NumPy product, on two calls in a row (the second smaller, so stale scratch contents of the
first call would show), plus the host-side rejection of a product too large for the fixed
scratch."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_gram_noalloc_matches_gram_on_consecutive_calls():
    import torch
    from paper_2304_00337_amd import Solver, native, to_device_block
    s = Solver(16, 16, 1.0, 1.0, np.ones(256), nev=2, nthrow=0)
    rng = np.random.default_rng(21)
    for length, q, r in ((70000, 24, 40), (3001, 5, 7)):
        X = rng.standard_normal((length, q)) + 1j * rng.standard_normal((length, q))
        W = rng.standard_normal((length, r)) + 1j * rng.standard_normal((length, r))
        Xd, Wd = to_device_block(X), to_device_block(W)
        ref = s.gram(Xd, Wd)
        out = torch.full((q * r * 2,), float("nan"), dtype=torch.float64, device="cuda")
        s.gram_noalloc(Xd, Wd, out)
        torch.cuda.synchronize()
        g = out.cpu().numpy().reshape(q, r, 2)
        got = g[..., 0] + 1j * g[..., 1]
        print(f"len {length} q {q} r {r}: max |noalloc - gram| {np.abs(got - ref).max():.1e}", flush=True)
        assert np.array_equal(got, ref)
        exact = X.conj().T @ W
        assert np.abs(got - exact).max() <= 1e-13 * np.abs(exact).max() * np.sqrt(length)
    # row blocks x q x r x 2 above 2^21 doubles: rejected before anything is launched
    lib = native.load()
    dummy = torch.zeros(16, dtype=torch.float64, device="cuda")
    p = ctypes.c_void_p(dummy.data_ptr())
    rc = lib.bl_gram_noalloc(s.h, p, 70, p, 70, 300000, p)
    assert rc == native.BL_EINVAL
    s.close()
