"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module builds *inputs only*: raw site tensors, Hamiltonian matrices and the
classical Ising weight tensors.  It holds none of the CTMRG arithmetic (no C4v
average, no double layer, no boundary tensors, no renormalisation); both the
oracle and the HIP path receive what is built here and do that work themselves.

Recipes
-------
* Site tensor A[s,u,l,d,r] (legs: physical, up, left, down, right): i.i.d.
  N(0,1) entries from ``numpy.random.default_rng(seed).standard_normal``.  The
  C4v average and the max-abs normalisation are applied by the method itself
  (iPEPS paragraph, C4v footnote).
* Finite-difference probe entries: ``default_rng(seed + 1000).choice(d*D**4, n)``.
* Spin-1/2 bond Hamiltonians (J = 1, S = sigma/2) as real 4x4 matrices with the
  row index (s1, s2) and column index (s1', s2'), s = 0 meaning spin up.
  ``heisenberg_bond_rotated`` is S.S after the pi rotation about y on one
  sublattice (Heisenberg-results paragraph): (Sx, Sy, Sz) -> (-Sx, Sy, -Sz).
* 2D Ising model at coupling K = beta*J: bond Boltzmann matrix
  B[s, s'] = exp(K s s'), split symmetrically as B = W W with W = sqrt(B).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "random_site_tensor",
    "fd_entries",
    "pauli",
    "heisenberg_bond",
    "heisenberg_bond_rotated",
    "ising_sqrt_boltzmann",
    "ising_classical_tensor",
    "ising_impurity_tensor",
    "ising_boundary_vector",
    "ising_peps_tensor",
    "product_state_tensor",
]


def random_site_tensor(d: int, D: int, seed: int) -> np.ndarray:
    """Raw i.i.d. N(0,1) site tensor A[s,u,l,d,r], float64, C-contiguous."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.standard_normal((d, D, D, D, D)))


def fd_entries(d: int, D: int, seed: int, n: int = 32) -> np.ndarray:
    """Flat indices of A probed by central finite differences."""
    rng = np.random.default_rng(seed + 1000)
    return np.sort(rng.choice(d * D ** 4, size=n, replace=False))


def pauli():
    """(sx, sy, sz) with sy returned as the real matrix i*sigma_y = [[0,1],[-1,0]].

    sigma_y itself is imaginary; every bond operator used here contains it twice,
    so sy (x) sy = -(i sy) (x) (i sy) is real.
    """
    sx = np.array([[0.0, 1.0], [1.0, 0.0]])
    isy = np.array([[0.0, 1.0], [-1.0, 0.0]])
    sz = np.array([[1.0, 0.0], [0.0, -1.0]])
    return sx, isy, sz


def heisenberg_bond() -> np.ndarray:
    """S_i . S_j for spin 1/2 as a real 4x4 matrix (eigenvalues -3/4, 1/4 x3)."""
    sx, isy, sz = pauli()
    return 0.25 * (np.kron(sx, sx) - np.kron(isy, isy) + np.kron(sz, sz))


def heisenberg_bond_rotated() -> np.ndarray:
    """S_i . S_j with site j rotated by exp(i pi sigma_y / 2): 1/4(-XX + YY - ZZ)."""
    sx, isy, sz = pauli()
    return 0.25 * (-np.kron(sx, sx) - np.kron(isy, isy) - np.kron(sz, sz))


def ising_sqrt_boltzmann(K: float) -> np.ndarray:
    """W = sqrt(B), B = [[e^K, e^-K], [e^-K, e^K]] (symmetric square root).

    B has eigenvectors (1, 1)/sqrt2 and (1, -1)/sqrt2 with eigenvalues 2cosh K
    and 2sinh K; W takes their square roots (K >= 0).
    """
    lp = np.sqrt(2.0 * np.cosh(K))
    lm = np.sqrt(2.0 * np.sinh(K)) if K > 0 else 0.0
    pp = 0.5 * np.array([[1.0, 1.0], [1.0, 1.0]])
    pm = 0.5 * np.array([[1.0, -1.0], [-1.0, 1.0]])
    return lp * pp + lm * pm


def _four_leg(W: np.ndarray, weight: np.ndarray) -> np.ndarray:
    # t[u,l,d,r] = sum_s weight[s] W[s,u] W[s,l] W[s,d] W[s,r]
    t = np.zeros((2, 2, 2, 2))
    for s in range(2):
        t += weight[s] * np.einsum("u,l,d,r->uldr", W[s], W[s], W[s], W[s])
    return t


def ising_classical_tensor(K: float) -> np.ndarray:
    """Classical Ising weight tensor a[u,l,d,r] (bond 2); its network is Z(K)."""
    return _four_leg(ising_sqrt_boltzmann(K), np.array([1.0, 1.0]))


def ising_impurity_tensor(K: float) -> np.ndarray:
    """Same as the weight tensor with the spin value inserted: sum_s s * (...)."""
    return _four_leg(ising_sqrt_boltzmann(K), np.array([1.0, -1.0]))


def ising_boundary_vector(K: float, biased: bool = False) -> np.ndarray:
    """Vector contracted with each open leg of the Ising network at the boundary.

    Unbiased: all ones (free boundary).  Biased: W^{-1} e_up, which fixes every
    boundary spin up (used below the critical temperature to select one of the
    two ordered states).
    """
    if not biased:
        return np.ones(2)
    W = ising_sqrt_boltzmann(K)
    return np.linalg.solve(W, np.array([1.0, 0.0]))


def ising_peps_tensor(K: float) -> np.ndarray:
    """Rank-5 site tensor A[s,u,l,d,r] = V[s,u]V[s,l]V[s,d]V[s,r], V = sqrt(B(K/2)).

    The state psi(sigma) = prod_bonds exp((K/2) s s') has norm <psi|psi> = Z(K),
    so its double-layer network is the Ising partition function at coupling K.
    """
    V = ising_sqrt_boltzmann(0.5 * K)
    A = np.zeros((2, 2, 2, 2, 2))
    for s in range(2):
        A[s] = np.einsum("u,l,d,r->uldr", V[s], V[s], V[s], V[s])
    return A


def product_state_tensor(psi, D: int) -> np.ndarray:
    """Product state embedded at bond dimension D: only the virtual index 0 is used."""
    psi = np.asarray(psi, dtype=np.float64)
    A = np.zeros((psi.size, D, D, D, D))
    A[:, 0, 0, 0, 0] = psi
    return A
