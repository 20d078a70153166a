"""Write the oracle's figures for QR-CTMRG cases too large to run in a test.

Calls only the FP64 oracle (oracle/) and the seeded inputs (synth/).  For
each case (d = 2, seeded random C4v tensor):

* A prepared and doubled (a1, a2); the boundary initialisation and the one
  standard warm-up step (a3, a4), with the gap of the warm-up's enlarged-corner
  spectrum at the chi cut (a cut through a degenerate pair would leave the
  kept subspace undefined);
* a few QR-CTMRG steps (a5-a10): the spectrum change of each step, the corner
  spectrum after the last one, and the energy after each step (a11): the
  nearest-neighbour Heisenberg energy (sublattice-rotated bond), plus 2 J2 <S.S>
  of the diagonal pair for the J1-J2 cases (J1-J2 paragraph);
* dE/dA through k tracked QR steps from that environment (a12): the energy
  E_k, the gradient's norm, its entries at 64 seeded positions (all entries for
  the smaller cases), and the two invariants of the exact gradient.

Run from the repository root:  python tests/golden/make_qrctm_golden.py CASE...
(no CASE: all).  The D = 8 case needs about 40 GB of memory and half an hour
on 8 cores; the others take seconds to minutes.
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

HERE = os.path.dirname(os.path.abspath(__file__))
CITE = ("oracle/ (FP64) via tests/golden/make_qrctm_golden.py; QR-CTMRG paragraph (reduced corner, "
        "QR, T' and accelerated corner), standard-CTMRG paragraph and its footnote "
        "(initialisation, warm-up), Heisenberg and J1-J2 paragraphs (energy), AD paragraph "
        "(k tracked steps)")

# name: (D, chi, QR steps, tracked steps k (None: no gradient), J2, store every gradient entry)
CASES = {
    "qrctm_d2_D6_chi144": (6, 144, 3, 10, 0.0, True),
    "qrctm_d2_D8_chi256": (8, 256, 3, 4, 0.0, False),
    "j1j2_d2_D6_chi72": (6, 72, 3, 2, 0.5, True),
    "j1j2_d2_D7_chi98": (7, 98, 3, None, 0.5, False),
    "j1j2_d2_D7_chi196": (7, 196, 3, 1, 0.5, False),
}
d, SEED = 2, 1


def log(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


def energy(C, T, As, h, h2, J2):
    if J2 != 0.0:
        return float(obs.energy_j1j2(C, T, As, h, h2, J2))
    return float(obs.energy_nn(C, T, As, h))


def run(name):
    D, chi, nqr, k, J2, full = CASES[name]
    log(f"{name}: D={D} chi={chi} QR steps {nqr} k {k} J2 {J2}")
    A = inp.random_site_tensor(d, D, SEED)
    As = ctm.prepare_site_tensor(A)
    a = ctm.double_layer(As)
    C, T = ctm.sym_norm(*ctm.init_env(a, ctm.identity_boundary_vector(D)))
    assert ctm.warmup_steps_needed(C.shape[0], D * D, chi) == 1
    lam = np.linalg.eigvalsh(ctm.enlarged_corner(C, T, a))
    mags = np.sort(np.abs(lam))[::-1]
    cut_gap = float((mags[chi - 1] - mags[chi]) / mags[0])
    log(f"cut gap {cut_gap:.3e}")
    C, T = ctm.sym_norm(*ctm.eigh_step(C, T, a, chi))
    h, h2 = inp.heisenberg_bond_rotated(), inp.heisenberg_bond()
    s_prev = ctm.spectrum(C)
    deltas, energies = [], []
    for i in range(nqr):
        C, T = ctm.sym_norm(*ctm.qr_step(C, T, a))
        s = ctm.spectrum(C)
        deltas.append(float(ctm.spectrum_delta(s, s_prev)))
        s_prev = s
        energies.append(energy(C, T, As, h, h2, J2))
        log(f"QR step {i + 1}: delta {deltas[-1]:.6e} energy {energies[-1]:.15f}")
    out = {
        "cite": CITE, "d": d, "D": D, "chi": chi, "seed": SEED, "qr_steps": nqr, "k_tracked": k,
        "J2": J2, "h_nn": "sublattice-rotated Heisenberg bond (synth.inputs.heisenberg_bond_rotated)",
        "h_nnn": "Heisenberg bond S.S (synth.inputs.heisenberg_bond)" if J2 else None,
        "warmup_cut_gap_rel": cut_gap, "deltas": deltas, "energies": energies,
        "spectrum_top64": [float(x) for x in s_prev[:64]], "spectrum_len": int(s_prev.size),
    }
    if k is not None:
        log(f"gradient, k = {k}")
        e_k, g = adj.energy_grad_k(A, C, T, k, h, h2 if J2 else None, J2)
        gf = g.ravel()
        idx = np.arange(gf.size) if full else inp.fd_entries(d, D, SEED, n=64)
        out.update({
            "energy_k": float(e_k),
            "grad_norm": float(np.linalg.norm(gf)),
            "grad_dot_A": float(np.dot(gf, A.ravel())),
            "grad_c4v_residual": float(np.abs(ctm.c4v_average(g) - g).max()),
            "grad_entries_index": [int(i) for i in idx],
            "grad_entries": [float(gf[i]) for i in idx],
        })
        log(f"E_k {e_k:.15f} |g| {np.linalg.norm(gf):.6e}")
    path = os.path.join(HERE, name + ".json")
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
    log(f"wrote {path}")


if __name__ == "__main__":
    for name in sys.argv[1:] or list(CASES):
        run(name)
