"""ctm_qr_noalloc (the QR entry point with the library's fixed scratch) against
ctm_qr (caller workspace), through the C ABI: two calls in a row, the second
with a smaller input, then a rank-deficient one (the Householder fallback in
the same scratch); sizes beyond the fixed scratch are refused before any GPU
work.  Same kernels and scratch layout on both sides, so the results are
bitwise equal (integer-exact bar)."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_2505_00494_amd as P  # noqa: E402
from paper_2505_00494_amd import qrctm as B  # noqa: E402


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda:0")


def test_qr_noalloc_matches_workspace_qr():
    rng = np.random.default_rng(11)
    cases = [("large", rng.standard_normal((5184, 144))),
             ("smaller", rng.standard_normal((1000, 37)))]
    M = rng.standard_normal((300, 24))
    M[:, 5] = 0.0
    M[:, 9] = M[:, 2]
    cases.append(("rank deficient", M))
    for name, Mh in cases:
        print(f"no-alloc QR {name} {Mh.shape}", flush=True)
        Md = _dev(Mh)
        Qw, Rw, uw = P.qr(Md, return_used=True)
        Qn, Rn, un = P.qr_noalloc(Md, return_used=True)
        torch.cuda.synchronize()
        assert un == uw, name
        assert torch.equal(Qn, Qw) and torch.equal(Rn, Rw), name
        Q, R = Qn.cpu().numpy(), Rn.cpu().numpy()
        n = Mh.shape[1]
        assert np.abs(Q.T @ Q - np.eye(n)).max() < 1e-12
        assert np.abs(Q @ R - Mh).max() < 1e-12 * max(1.0, np.abs(Mh).max())
    assert cases and un  # the last case ran the Householder kernel


def test_qr_noalloc_refuses_oversized_input():
    L = P.lib()
    m, n = 16384, 256
    assert L.ctm_qr_workspace_bytes(m, n) > L.ctm_qr_noalloc_max_bytes()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: refused before any GPU work
    rc = L.ctm_qr_noalloc(fake, fake, fake, m, n, 0, None, None)
    assert rc == B.CTM_EWORKSPACE
    assert b"fixed" in L.ctm_last_error(None)
