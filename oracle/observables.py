"""Oracle observables from a converged C4v environment, FP64 on the CPU.

TEST INFRASTRUCTURE ONLY (see the package docstring).

* Two-site reduced density matrix of a nearest-neighbour bond from the 2x1
  cluster (4 corners, 6 edges, two open sites) and the energy per site
  e = 2 Tr(rho h) / Tr rho (two bonds per site; Heisenberg-results paragraph,
  with h already sublattice-rotated by the caller).
* Next-nearest-neighbour (diagonal) reduced density matrix from the 2x2
  plaquette (four enlarged corners, two open diagonal sites), for the J1-J2
  model (J1-J2 paragraph): e = 2<h_nn> + 2 J2 <h_nnn>.
* Classical networks (Discussion paragraph: QR-CTMRG also applies to classical
  2D partition functions): ln kappa per site from the 3x3, 2x2 and 3x2
  networks, and one-site expectation values with an impurity tensor.
"""
from __future__ import annotations

import numpy as np

from .ctmrg import open_double_layer


def _left_column(C, T):
    # E1[q, L, t] = sum C[q,p] T[p,L,r] C[r,t]; corner legs toward the top/bottom
    # edges are q and t, the edge's inward leg L faces the open site.
    F = np.tensordot(C, T, axes=([1], [0]))             # [q,L,r]
    return np.tensordot(F, C, axes=([2], [0]))          # [q,L,t]


def half_cluster(C, T, A):
    """Left half of the 2x1 cluster with site 1 open.

    Left[q2, R, t2, s, s']: q2 / t2 are the top / bottom edge legs toward site 2,
    R the paired right leg of site 1, (s, s') the ket / bra physical legs.
    """
    E1 = _left_column(C, T)                                        # [q,L,t]
    E2 = np.einsum("qUw,qLt->wULt", T, E1, optimize=True)          # top edge
    ao = open_double_layer(A)                                      # [s,s',U,L,Dn,R]
    E3 = np.einsum("wULt,xyULDR->wtxyDR", E2, ao, optimize=True)
    Left = np.einsum("wtxyDR,tDv->wRvxy", E3, T, optimize=True)    # bottom edge
    return Left


def rdm_nn(C, T, A):
    """rho[s1, s1', s2, s2'] of a horizontal nearest-neighbour bond.

    The right half equals the left half (mirror symmetry of the C4v network),
    so rho = sum Left[.., s1, s1'] Left[.., s2, s2'].
    """
    Left = half_cluster(C, T, A)
    return np.einsum("wRvab,wRvcd->abcd", Left, Left, optimize=True)


def bond_expectation(rho, h):
    """<h> = Tr(rho h) / Tr rho with rho[s1,s1',s2,s2'] and h[(s1 s2),(s1' s2')]."""
    d = rho.shape[0]
    rm = rho.transpose(0, 2, 1, 3).reshape(d * d, d * d)   # [(s1 s2),(s1' s2')]
    return float(np.trace(rm @ h) / np.trace(rm))


def energy_nn(C, T, A, h):
    """Energy per site of a nearest-neighbour model: 2 <h_bond>."""
    return 2.0 * bond_expectation(rdm_nn(C, T, A), h)


# ----------------------------------------------------------------------------
# 2x2 plaquette, diagonal pair (top-left and bottom-right sites open).
# ----------------------------------------------------------------------------


def enlarged_corner_open(C, T, A):
    """Enlarged corner with its site open: Co[s, s', (e,dn), (c,r)].

    Same contraction as the enlarged corner of the standard step, with the
    open double layer in place of a.
    """
    chi, Dab, _ = T.shape
    ct3 = (C @ T.reshape(chi, Dab * chi)).reshape(chi, Dab, chi)   # [y,u,c]
    G = np.tensordot(T, ct3, axes=([0], [0]))                      # [l,e,u,c]
    ao = open_double_layer(A)                                      # [s,s',U,L,Dn,R]
    Co = np.tensordot(G, ao, axes=([0, 2], [3, 2]))                # [e,c,s,s',dn,r]
    Co = Co.transpose(2, 3, 0, 4, 1, 5)                            # [s,s',e,dn,c,r]
    d = A.shape[0]
    return Co.reshape(d, d, chi * Dab, chi * Dab)


def enlarged_corner_closed(C, T, A):
    from .ctmrg import double_layer, enlarged_corner
    return enlarged_corner(C, T, double_layer(A))


def rdm_nnn(C, T, A):
    """rho[s1, s1', s2, s2'] of a diagonal pair from the 2x2 plaquette.

    The plaquette is the cyclic product of four enlarged corners; by C4v all four
    are the same matrix (symmetric), so with two open diagonal corners
    rho = Tr(Co1 Cc Co2 Cc).
    """
    Co = enlarged_corner_open(C, T, A)
    Co = 0.5 * (Co + Co.transpose(0, 1, 3, 2))
    Cc = enlarged_corner_closed(C, T, A)
    X = np.einsum("abij,jk->abik", Co, Cc, optimize=True)          # Co1 Cc
    return np.einsum("abij,cdji->abcd", X, X, optimize=True)


def energy_j1j2(C, T, A, h_nn, h_nnn, J2):
    """Energy per site: 2 <h_nn> + 2 J2 <h_nnn> (two NN and two NNN bonds per site)."""
    e1 = 2.0 * bond_expectation(rdm_nn(C, T, A), h_nn)
    e2 = 2.0 * J2 * bond_expectation(rdm_nnn(C, T, A), h_nnn)
    return e1 + e2


# ----------------------------------------------------------------------------
# Classical networks.
# ----------------------------------------------------------------------------


def z33(C, T, a):
    E1 = _left_column(C, T)                                        # [q,L,t]
    E2 = np.einsum("qUw,qLt->wULt", T, E1, optimize=True)
    E3 = np.einsum("wULt,ULDR->wtDR", E2, a, optimize=True)
    Left = np.einsum("wtDR,tDv->wRv", E3, T, optimize=True)
    return float(np.einsum("wRv,wRv->", Left, E1))


def z22(C):
    return float(np.trace(C @ C @ C @ C))


def z32(C, T):
    E1 = _left_column(C, T)
    return float(np.sum(E1 * E1))


def ln_kappa(C, T, a):
    """ln of the partition function per site: ln Z33 + ln Z22 - 2 ln Z32."""
    return float(np.log(z33(C, T, a)) + np.log(z22(C)) - 2.0 * np.log(z32(C, T)))


def expect_site(C, T, a, impurity):
    """<O> at one site: network with the impurity tensor / network with a."""
    return z33(C, T, impurity) / z33(C, T, a)
