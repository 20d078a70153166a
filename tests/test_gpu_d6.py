"""Forward and adjoint at the benchmark size d = 2, D = 6, chi = 144.

* Against figures the oracle stored (tests/golden/qrctm_d2_D6_chi144.json,
  written by tests/golden/make_qrctm_golden.py, which calls only oracle/ and
  synth/): both sides start from the seeded tensor, run their own warm-up
  (the kept subspace has a relative gap of 3.6e-5 at the chi cut, so it is
  the same) and three QR steps; spectrum changes and energies agree to
  1e-10, and dE/dA through k = 10 tracked steps (the benchmark's gradient)
  agrees with the oracle's reverse mode entry by entry to 1e-9 in norm.
* Against central differences of the GPU's own forward pass on 32 seeded
  entries of A (the differentiated function E_k(P(A); C0, T0), k = 10).  The
  energy after ten steps carries a rounding noise of a few 1e-15 (tens of
  ulps; the step map amplifies rounding), so a central difference has a noise
  floor of about that over 2h: at h = 1e-6 it is ~1e-6 of the gradient
  entries (measured 1.25e-6), at h = 1e-5 ten times less, with the truncation
  error (h^2) still far below.  The check is 1e-6 at h = 1e-5, and 2.5e-6 at
  h = 1e-6 (the noise floor plus margin).
"""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_2505_00494_amd as P  # noqa: E402
from oracle import ctmrg as ctm  # noqa: E402
from synth import inputs as inp  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "qrctm_d2_D6_chi144.json")
H = inp.heisenberg_bond_rotated()


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda:0")


def _golden():
    with open(GOLDEN) as f:
        return json.load(f)


@pytest.mark.parametrize("split", [1, 0])
def test_d6_chi144_gradient_matches_oracle(split):
    g = _golden()
    d, D, chi, k = g["d"], g["D"], g["chi"], g["k_tracked"]
    print(f"d={d} D={D} chi={chi} k={k} edge_split={split}", flush=True)
    A = inp.random_site_tensor(d, D, g["seed"])
    ctx = P.Context(_dev(A), chi, k_tracked=k, edge_split=split)
    for i in range(g["qr_steps"]):
        dl = ctx.step(1)
        e = ctx.energy(H)
        assert abs(dl - g["deltas"][i]) < 1e-10 * g["deltas"][i], i
        assert abs(e - g["energies"][i]) < 1e-10 * abs(g["energies"][i]), i
    s = ctx.spectrum()
    assert np.abs(s[:64] - np.array(g["spectrum_top64"])).max() < 1e-12
    ek, gA = ctx.energy_grad(H)
    assert abs(ek - g["energy_k"]) < 1e-10 * abs(g["energy_k"])
    gf = gA.cpu().numpy().ravel()
    ref = np.zeros_like(gf)
    ref[np.array(g["grad_entries_index"])] = np.array(g["grad_entries"])
    assert np.linalg.norm(gf - ref) / np.linalg.norm(ref) < 1e-9
    assert abs(np.dot(gf, A.ravel())) < 1e-10 * np.linalg.norm(gf) * np.linalg.norm(A)
    ctx.close()


def test_d6_chi144_gradient_matches_gpu_finite_differences():
    g = _golden()
    d, D, chi, k, seed = g["d"], g["D"], g["chi"], g["k_tracked"], g["seed"]
    A = inp.random_site_tensor(d, D, seed)
    ctx = P.Context(_dev(A), chi, k_tracked=k)
    ctx.step(g["qr_steps"])
    C0, T0 = ctx.get_env()
    _, gA = ctx.energy_grad(H)
    gf = gA.cpu().numpy().ravel()

    def energy(Ax):
        ctx.set_tensor(_dev(Ax))
        ctx.set_env(C0, T0)
        ctx.step(k)
        return ctx.energy(H)

    idx = inp.fd_entries(d, D, seed, n=32)
    for h, bar in ((1e-5, 1e-6), (1e-6, 2.5e-6)):
        fd = []
        for i in idx:
            Ap, Am = A.ravel().copy(), A.ravel().copy()
            Ap[i] += h
            Am[i] -= h
            fd.append((energy(Ap.reshape(A.shape)) - energy(Am.reshape(A.shape))) / (2 * h))
        fd = np.array(fd)
        err = np.linalg.norm(fd - gf[idx]) / np.linalg.norm(gf[idx])
        print(f"FD (32 entries, h = {h:.0e}) relative error {err:.3e}", flush=True)
        assert err < bar, h
    ctx.close()
