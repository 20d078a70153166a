"""Forward and adjoint at d = 2, D = 8, chi = 256 against the oracle's figures.

The oracle needs half an hour and ~40 GB at this size, so its results are
stored in tests/golden/qrctm_d2_D8_chi256.json by
tests/golden/make_qrctm_golden.py (which calls only oracle/ and synth/):
three QR steps after the warm-up, then dE/dA through k = 4 tracked steps.  Both sides start from the same seeded
tensor and run their own initialisation and warm-up step; the warm-up keeps
the 256 largest |lambda| of a 4096 x 4096 enlarged corner, whose spectrum has
a relative gap of 2e-5 at the cut, so the kept subspace is the same and the
environments agree up to a gauge.  Only gauge-invariant figures are compared:
spectrum changes, energies, the corner spectrum and dE/dA.
Tolerances: energy 1e-9 relative, dE/dA 1e-6 relative.
"""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_2505_00494_amd as P  # noqa: E402
from synth import inputs as inp  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "qrctm_d2_D8_chi256.json")


@pytest.mark.parametrize("split", [1, 0])
def test_d8_chi256_forward_and_gradient_match_oracle(split):
    with open(GOLDEN) as f:
        g = json.load(f)
    d, D, chi = g["d"], g["D"], g["chi"]
    print(f"d={d} D={D} chi={chi} edge_split={split}: warm-up", flush=True)
    A = inp.random_site_tensor(d, D, g["seed"])
    h = inp.heisenberg_bond_rotated()
    ctx = P.Context(torch.as_tensor(A, device="cuda:0"), chi, k_tracked=g["k_tracked"],
                    edge_split=split)
    for i in range(g["qr_steps"]):
        dl = ctx.step(1)
        e = ctx.energy(h)
        print(f"step {i + 1}: delta {dl:.6e} energy {e:.15f}", flush=True)
        assert abs(dl - g["deltas"][i]) < 1e-9 * g["deltas"][i], i
        assert abs(e - g["energies"][i]) < 1e-9 * abs(g["energies"][i]), i
    s = ctx.spectrum()
    assert s.size == g["spectrum_len"]
    assert np.abs(s[:64] - np.array(g["spectrum_top64"])).max() < 1e-11
    print("gradient", flush=True)
    ek, gA = ctx.energy_grad(h)
    assert abs(ek - g["energy_k"]) < 1e-9 * abs(g["energy_k"])
    gf = gA.cpu().numpy().ravel()
    ref = np.array(g["grad_entries"])
    got = gf[np.array(g["grad_entries_index"])]
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-6
    assert abs(np.linalg.norm(gf) - g["grad_norm"]) < 1e-6 * g["grad_norm"]
    # invariants of the exact gradient (scale invariance, C4v symmetry)
    assert abs(np.dot(gf, A.ravel())) < 1e-10 * np.linalg.norm(gf) * np.linalg.norm(A)
    ctx.close()
