"""Write the oracle's figures for QR-CTMRG at d = 2, D = 8, chi = 256.

Calls only the FP64 oracle (oracle/) and the seeded inputs (synth/):

* A: the seeded random C4v tensor (seed 1), prepared and doubled (a1, a2);
* the boundary initialisation and the standard warm-up step (a3, a4), with
  the gap of the warm-up's enlarged-corner spectrum at the chi cut (a cut
  through a degenerate pair would leave the kept subspace undefined);
* three QR-CTMRG steps (a5-a10): the spectrum change of each step, the corner
  spectrum after the last one, and the nearest-neighbour Heisenberg energy
  (sublattice-rotated bond) after each step (a11);
* dE/dA through k = 1 tracked QR step from that environment (a12): the energy
  E_k, the gradient's norm and its entries at 64 seeded positions, and the two
  invariants of the exact gradient.

Run from the repository root:  python tests/golden/make_qrctm_d8_golden.py
It needs about 40 GB of memory and a few minutes on 8 cores.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import adjoint as adj  # noqa: E402
from oracle import ctmrg as ctm  # noqa: E402
from oracle import observables as obs  # noqa: E402
from synth import inputs as inp  # noqa: E402

d, D, CHI, SEED, NQR, K = 2, 8, 256, 1, 3, 1
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "qrctm_d2_D8_chi256.json")


def log(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


def main():
    A = inp.random_site_tensor(d, D, SEED)
    As = ctm.prepare_site_tensor(A)
    a = ctm.double_layer(As)
    log("init")
    C, T = ctm.sym_norm(*ctm.init_env(a, ctm.identity_boundary_vector(D)))
    assert ctm.warmup_steps_needed(C.shape[0], D * D, CHI) == 1
    log("warm-up: enlarged corner and its spectrum")
    lam = np.linalg.eigvalsh(ctm.enlarged_corner(C, T, a))
    mags = np.sort(np.abs(lam))[::-1]
    cut_gap = float((mags[CHI - 1] - mags[CHI]) / mags[0])
    log(f"cut gap {cut_gap:.3e}")
    C, T = ctm.sym_norm(*ctm.eigh_step(C, T, a, CHI))
    h = inp.heisenberg_bond_rotated()
    s_prev = ctm.spectrum(C)
    deltas, energies = [], []
    for i in range(NQR):
        log(f"QR step {i + 1}")
        C, T = ctm.sym_norm(*ctm.qr_step(C, T, a))
        s = ctm.spectrum(C)
        deltas.append(float(ctm.spectrum_delta(s, s_prev)))
        s_prev = s
        energies.append(float(obs.energy_nn(C, T, As, h)))
        log(f"  delta {deltas[-1]:.6e} energy {energies[-1]:.15f}")
    log(f"gradient, k = {K}")
    e_k, g = adj.energy_grad_k(A, C, T, K, h)
    idx = inp.fd_entries(d, D, SEED, n=64)
    gf = g.ravel()
    out = {
        "cite": "oracle/ (FP64) via tests/golden/make_qrctm_d8_golden.py; QR-CTMRG paragraph "
                "(reduced corner, QR, T' and accelerated corner), standard-CTMRG paragraph and its "
                "footnote (initialisation, warm-up), Heisenberg paragraph (energy), AD paragraph "
                "(k tracked steps)",
        "d": d, "D": D, "chi": CHI, "seed": SEED, "qr_steps": NQR, "k_tracked": K,
        "warmup_cut_gap_rel": cut_gap,
        "deltas": deltas,
        "energies": energies,
        "spectrum_top64": [float(x) for x in s_prev[:64]],
        "spectrum_len": int(s_prev.size),
        "energy_k": float(e_k),
        "grad_norm": float(np.linalg.norm(gf)),
        "grad_dot_A": float(np.dot(gf, A.ravel())),
        "grad_c4v_residual": float(np.abs(ctm.c4v_average(g) - g).max()),
        "grad_entries_index": [int(i) for i in idx],
        "grad_entries": [float(gf[i]) for i in idx],
    }
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    log(f"wrote {OUT}")


if __name__ == "__main__":
    main()
