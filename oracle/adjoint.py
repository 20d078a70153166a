"""Oracle reverse mode: dE/dA through k tracked QR-CTMRG steps, FP64 on the CPU.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The differentiated function (automatic-differentiation paragraph: untracked
steps, then k steps with gradient tracking, then the energy) is

    E(A) = e( C_k, T_k, As ),  As = P(A) / max|P(A)|,  a = sum_s As (x) As,
    (C_{i+1}, T_{i+1}) = sym_norm( QR-step(C_i, T_i, a) ),  (C_0, T_0) held fixed,

with e the nearest-neighbour energy 2<h>, or the J1-J2 energy 2<h> + 2 J2 <h_nnn>
(J1-J2 paragraph; the diagonal pair from the 2x2 plaquette).

Every adjoint below is written by hand from the forward formula it reverses.
The QR adjoint (thin QR, m >= n, diag R > 0) is
    Abar = (Qbar + Q copyltu(M)) R^{-T},  M = R Rbar^T - Qbar^T Q,
    copyltu(M) = tril(M) + tril(M, -1)^T,
the form used in the AD literature the paper cites for iPEPS (Liao et al. 2019).
"""
from __future__ import annotations

import numpy as np

from . import ctmrg as ctm
from . import observables as obs


def einsum_vjp(spec: str, X: np.ndarray, Y: np.ndarray, Zbar: np.ndarray):
    """Cotangents of Z = einsum(spec, X, Y) (each index once per operand)."""
    ins, out = spec.split("->")
    sx, sy = ins.split(",")
    Xbar = np.einsum(f"{out},{sy}->{sx}", Zbar, Y, optimize=True)
    Ybar = np.einsum(f"{sx},{out}->{sy}", X, Zbar, optimize=True)
    return Xbar, Ybar


def copyltu(M: np.ndarray) -> np.ndarray:
    return np.tril(M) + np.tril(M, -1).T


def regularized_inverse(R, eps_rel):
    """Inverse of the upper-triangular R by back substitution in which each
    division by R_ii becomes a product with d_i = R_ii / (R_ii^2 + eps^2),
    eps = eps_rel max|R_ii| (Tikhonov form of 1/R_ii).  With N the strictly
    upper part of R and Dl = diag(d), the substitution R x = e_j reads
    x = Dl (e_j - N x), so the result is (I + Dl N)^{-1} Dl; eps_rel = 0 gives
    R^{-1}."""
    r = np.diag(R)
    eps = eps_rel * np.abs(r).max()
    dl = np.diag(r / (r * r + eps * eps))
    n = R.shape[0]
    return np.linalg.solve(np.eye(n) + dl @ np.triu(R, 1), dl)


def qr_backward(Q, R, Qbar, Rbar, eps_rel=0.0):
    M = R @ Rbar.T - Qbar.T @ Q
    B = Qbar + Q @ copyltu(M)
    if eps_rel > 0.0:
        return B @ regularized_inverse(R, eps_rel).T
    # B R^{-T}: solve R X^T = B^T
    return np.linalg.solve(R, B.T).T


# ----------------------------------------------------------------------------
# a9 / symmetrisation adjoints
# ----------------------------------------------------------------------------


def norm_backward(X, Xbar):
    """y = X/||X||  ->  Xbar_in = (ybar - y <y, ybar>) / ||X||."""
    nrm = np.linalg.norm(X)
    y = X / nrm
    return (Xbar - y * np.sum(y * Xbar)) / nrm


def sym_norm_backward(Cp, Tp, Cbar, Tbar):
    Cs = 0.5 * (Cp + Cp.T)
    Ts = 0.5 * (Tp + Tp.transpose(2, 1, 0))
    Csb = norm_backward(Cs, Cbar)
    Tsb = norm_backward(Ts, Tbar)
    return 0.5 * (Csb + Csb.T), 0.5 * (Tsb + Tsb.transpose(2, 1, 0))


# ----------------------------------------------------------------------------
# One QR step, reversed.
# ----------------------------------------------------------------------------


def qr_step_backward(C, T, a, Cnbar, Tnbar, eps_rel=0.0):
    """Given the step's inputs and cotangents of its normalised outputs,
    return (Cbar, Tbar, abar); eps_rel > 0 regularises R^{-1} of the QR adjoint."""
    chi, Dab, _ = T.shape
    p = ctm.qr_step_parts(C, T, a)
    Q, R, Y, Z, Tp, Cp = p["Q"], p["R"], p["Y"], p["Z"], p["Tp"], p["Cp"]
    chin = Q.shape[1]
    Q3 = Q.reshape(chi, Dab, chin)

    Cpb, Tpb = sym_norm_backward(Cp, Tp, Cnbar, Tnbar)

    # a8: W = R . Q3 ; C' = T'^T-contract W
    W = np.tensordot(R, Q3, axes=([1], [0]))                        # [g,r,b]
    Tpb2, Wb = einsum_vjp("gra,grb->ab", Tp, W, Cpb)
    Tpb = Tpb + Tpb2
    Rb, Q3b = einsum_vjp("gc,crb->grb", R, Q3, Wb)

    # a7 (3c): T'[a,r,b] = Z[a,f,d,r] Q3[f,d,b]
    Zb, Q3b2 = einsum_vjp("afdr,fdb->arb", Z, Q3, Tpb)
    Q3b = Q3b + Q3b2
    # a7 (3b): Z[a,f,d,r] = Y[a,u,l,f] a[u,l,d,r]
    Yb, ab = einsum_vjp("aulf,uldr->afdr", Y, a, Zb)
    # a7 (3a): Y[a,u,l,f] = Q3[e,u,a] T[e,l,f]
    Q3b3, Tb = einsum_vjp("eua,elf->aulf", Q3, T, Yb)
    Q3b = Q3b + Q3b3

    # a6: QR
    ctb = qr_backward(Q, R, Q3b.reshape(chi * Dab, chin), Rb, eps_rel)

    # a5: ct = C . T (as chi x (Dab chi))
    ctb2 = ctb.reshape(C.shape[0], Dab * T.shape[2])
    Tmat = T.reshape(chi, Dab * T.shape[2])
    Cb = ctb2 @ Tmat.T
    Tb = Tb + (C.T @ ctb2).reshape(T.shape)
    return Cb, Tb, ab


# ----------------------------------------------------------------------------
# Energy (2x1 cluster), reversed.
# ----------------------------------------------------------------------------


def energy_nn_backward(C, T, A, h):
    """Return (e, Cbar, Tbar, Abar_open) for e = 2 Tr(rho h)/Tr rho."""
    d = A.shape[0]
    F = np.tensordot(C, T, axes=([1], [0]))                          # [q,L,r]
    E1 = np.tensordot(F, C, axes=([2], [0]))                         # [q,L,t]
    E2 = np.einsum("qUw,qLt->wULt", T, E1, optimize=True)
    ao = ctm.open_double_layer(A)
    E3 = np.einsum("wULt,xyULDR->wtxyDR", E2, ao, optimize=True)
    Left = np.einsum("wtxyDR,tDv->wRvxy", E3, T, optimize=True)
    rho = np.einsum("wRvab,wRvcd->abcd", Left, Left, optimize=True)
    rm = rho.transpose(0, 2, 1, 3).reshape(d * d, d * d)
    num = float(np.trace(rm @ h))
    den = float(np.trace(rm))
    e = 2.0 * num / den

    rmb = (2.0 / den) * h.T - (2.0 * num / den ** 2) * np.eye(d * d)
    rhob = rmb.reshape(d, d, d, d).transpose(0, 2, 1, 3)
    Lb1, Lb2 = einsum_vjp("wRvab,wRvcd->abcd", Left, Left, rhob)
    Leftb = Lb1 + Lb2
    E3b, Tb = einsum_vjp("wtxyDR,tDv->wRvxy", E3, T, Leftb)
    E2b, aob = einsum_vjp("wULt,xyULDR->wtxyDR", E2, ao, E3b)
    Tb2, E1b = einsum_vjp("qUw,qLt->wULt", T, E1, E2b)
    Tb = Tb + Tb2
    Fb, Cb = einsum_vjp("qLr,rt->qLt", F, C, E1b)
    Cb2, Tb3 = einsum_vjp("qp,pLr->qLr", C, T, Fb)
    Cb = Cb + Cb2
    Tb = Tb + Tb3

    D = A.shape[1]
    aob8 = aob.reshape(d, d, D, D, D, D, D, D, D, D)  # [s,t,u,u',l,l',d,d',r,r']
    Ab = (np.einsum("staebfcgdh,tefgh->sabcd", aob8, A, optimize=True)
          + np.einsum("tsaebfcgdh,tabcd->sefgh", aob8, A, optimize=True))
    return e, Cb, Tb, Ab


def open_double_layer_backward(A, aobar):
    """Cotangent of A from that of a_open[s,t,(u u'),(l l'),(d d'),(r r')] =
    A[s,u,l,d,r] A[t,u',l',d',r'] (ket s, bra t)."""
    d, D = A.shape[0], A.shape[1]
    aob8 = aobar.reshape(d, d, D, D, D, D, D, D, D, D)  # [s,t,u,u',l,l',d,d',r,r']
    return (np.einsum("staebfcgdh,tefgh->sabcd", aob8, A, optimize=True)
            + np.einsum("tsaebfcgdh,tabcd->sefgh", aob8, A, optimize=True))


def _bond_rdm_bar(rho, h, scale):
    """(e, rhobar) for e = scale Tr(rm h) / Tr(rm), rm = rho as [(s1 s2),(s1' s2')]."""
    d = rho.shape[0]
    rm = rho.transpose(0, 2, 1, 3).reshape(d * d, d * d)
    num = float(np.trace(rm @ h))
    den = float(np.trace(rm))
    rmb = (scale / den) * h.T - (scale * num / den ** 2) * np.eye(d * d)
    return scale * num / den, rmb.reshape(d, d, d, d).transpose(0, 2, 1, 3)


def energy_nnn_backward(C, T, A, h, J2):
    """Return (e2, Cbar, Tbar, Abar) for the next-nearest-neighbour part
    e2 = 2 J2 Tr(rho h)/Tr rho of the J1-J2 energy, rho from the 2x2 plaquette
    (J1-J2 paragraph), reversing observables.rdm_nnn step by step:

        ct3[y,u,c]   = sum_x C[y,x] T[x,u,c]                 (reduced corner)
        G[l,e,u,c]   = sum_y T[y,l,e] ct3[y,u,c]
        Cc           = sym( G . a       -> [(e,dn),(c,r)] )  (closed enlarged corner)
        Co[s,t]      = sym( G . a_open  -> [(e,dn),(c,r)] )  (open enlarged corner)
        X[s,t]       = Co[s,t] Cc,   rho[s1,t1,s2,t2] = Tr(X[s1,t1] X[s2,t2]).
    """
    from .ctmrg import double_layer, open_double_layer
    d = A.shape[0]
    chi, Dab, _ = T.shape
    n = chi * Dab
    a = double_layer(A)
    ao = open_double_layer(A)
    ct3 = (C @ T.reshape(chi, Dab * chi)).reshape(chi, Dab, chi)
    G = np.einsum("yle,yuc->leuc", T, ct3, optimize=True)
    Ct4 = np.einsum("leuc,ulnr->ecnr", G, a, optimize=True)
    Cc = Ct4.transpose(0, 2, 1, 3).reshape(n, n)
    Cc = 0.5 * (Cc + Cc.T)
    Co6 = np.einsum("leuc,stulnr->stencr", G, ao, optimize=True)
    Co = Co6.reshape(d, d, n, n)
    Co = 0.5 * (Co + Co.transpose(0, 1, 3, 2))
    X = np.einsum("abij,jk->abik", Co, Cc, optimize=True)
    rho = np.einsum("abij,cdji->abcd", X, X, optimize=True)
    e2, rhob = _bond_rdm_bar(rho, h, 2.0 * J2)

    Xb = (np.einsum("abcd,cdji->abij", rhob, X, optimize=True)
          + np.einsum("cdab,cdji->abij", rhob, X, optimize=True))
    Cob = np.einsum("abik,jk->abij", Xb, Cc, optimize=True)       # Xb Cc^T
    Ccb = np.einsum("abij,abik->jk", Co, Xb, optimize=True)        # sum Co^T Xb
    Cob = 0.5 * (Cob + Cob.transpose(0, 1, 3, 2))
    Ccb = 0.5 * (Ccb + Ccb.T)
    Co6b = Cob.reshape(d, d, chi, Dab, chi, Dab)
    Gb1, aob = einsum_vjp("leuc,stulnr->stencr", G, ao, Co6b)
    Ct4b = Ccb.reshape(chi, Dab, chi, Dab).transpose(0, 2, 1, 3)
    Gb2, ab = einsum_vjp("leuc,ulnr->ecnr", G, a, Ct4b)
    Tb, ct3b = einsum_vjp("yle,yuc->leuc", T, ct3, Gb1 + Gb2)
    Cb, Tb2 = einsum_vjp("yx,xuc->yuc", C, T, ct3b)
    Ab = open_double_layer_backward(A, aob) + double_layer_backward(A, ab)
    return e2, Cb, Tb + Tb2, Ab


def energy_backward(C, T, A, h, h_nnn=None, J2=0.0):
    """(e, Cbar, Tbar, Abar) of e = 2 <h> (+ 2 J2 <h_nnn>) (observables.energy_j1j2)."""
    e, Cb, Tb, Ab = energy_nn_backward(C, T, A, h)
    if h_nnn is not None and J2 != 0.0:
        e2, Cb2, Tb2, Ab2 = energy_nnn_backward(C, T, A, h_nnn, J2)
        e, Cb, Tb, Ab = e + e2, Cb + Cb2, Tb + Tb2, Ab + Ab2
    return e, Cb, Tb, Ab


def double_layer_backward(A, abar):
    """a[(u u'),(l l'),(d d'),(r r')] = sum_s A[s,u,l,d,r] A[s,u',l',d',r']."""
    D = A.shape[1]
    ab8 = abar.reshape(D, D, D, D, D, D, D, D)        # [u,u',l,l',d,d',r,r']
    return (np.einsum("aebfcgdh,sefgh->sabcd", ab8, A, optimize=True)
            + np.einsum("aebfcgdh,sabcd->sefgh", ab8, A, optimize=True))


def prepare_backward(A_raw, Asbar):
    """As = P(A)/m, m = max|P(A)| (unique maximiser assumed)."""
    PA = ctm.c4v_average(A_raw)
    flat = np.abs(PA).ravel()
    i = int(np.argmax(flat))
    m = flat[i]
    sgn = np.sign(PA.ravel()[i])
    g = ctm.c4v_average(Asbar) / m
    coef = sgn * np.sum(Asbar * PA) / m ** 2
    ei = np.zeros(PA.size)
    ei[i] = 1.0
    g -= coef * ctm.c4v_average(ei.reshape(PA.shape))
    return g


# ----------------------------------------------------------------------------
# Checkpointed k-step gradient.
# ----------------------------------------------------------------------------


def _energy(C, T, As, h, h_nnn, J2):
    if h_nnn is not None and J2 != 0.0:
        return obs.energy_j1j2(C, T, As, h, h_nnn, J2)
    return obs.energy_nn(C, T, As, h)


def energy_k(A_raw, C0, T0, k, h, h_nnn=None, J2=0.0):
    """Forward only: E(A) as defined in the module docstring."""
    As = ctm.prepare_site_tensor(A_raw)
    a = ctm.double_layer(As)
    C, T = C0, T0
    for _ in range(k):
        C, T = ctm.sym_norm(*ctm.qr_step(C, T, a))
    return _energy(C, T, As, h, h_nnn, J2)


def energy_grad_k(A_raw, C0, T0, k, h, h_nnn=None, J2=0.0, qr_reg_eps=0.0):
    """(E, dE/dA_raw) with the k tracked steps reversed from stored (C_i, T_i);
    qr_reg_eps > 0 uses the regularised R^{-1} in every QR adjoint."""
    As = ctm.prepare_site_tensor(A_raw)
    a = ctm.double_layer(As)
    env = [(C0, T0)]
    C, T = C0, T0
    for _ in range(k):
        C, T = ctm.sym_norm(*ctm.qr_step(C, T, a))
        env.append((C, T))
    e, Cb, Tb, Asb = energy_backward(C, T, As, h, h_nnn, J2)
    ab = np.zeros_like(a)
    for i in range(k - 1, -1, -1):
        Ci, Ti = env[i]
        Cb, Tb, abi = qr_step_backward(Ci, Ti, a, Cb, Tb, qr_reg_eps)
        ab += abi
    Asb = Asb + double_layer_backward(As, ab)
    return e, prepare_backward(A_raw, Asb)


# ----------------------------------------------------------------------------
# Fixed-point (implicit) gradient at a converged environment.
# ----------------------------------------------------------------------------


def energy_grad_fixed_point(A_raw, C, T, h, tol=1e-12, max_iter=2000, h_nnn=None, J2=0.0):
    """(E, dE/dA_raw, n_iter) by differentiating the fixed-point condition.

    Discussion paragraph: the fixed-point AD scheme of Liao et al. (2019).
    Let F be one QR step followed by sym_norm.  A converged environment is a
    fixed point of F in C, but T can alternate between two gauges (a cycle of
    period 2), so the condition used is env* = G(env*, a) with G = F o F,
    which holds in either case.  The converged energy E(A) = e(env*(A), As(A))
    then has

        dE/dAs = de/dAs + lam . dG/da . da/dAs,
        lam    = ebar (I - dG/denv)^{-1} = sum_{n >= 0} ebar (dG/denv)^n,

    ebar = de/denv.  The series is summed term by term: each term reverses the
    two steps env* -> env1 = F(env*) -> env*, with the a-cotangent of every
    reversed step accumulated, until a term's norm falls below tol times that
    of ebar; it converges at the rate the CTMRG iteration itself does.
    n_iter counts the reversed steps (even); None means max_iter was reached.
    """
    As = ctm.prepare_site_tensor(A_raw)
    a = ctm.double_layer(As)
    C1, T1 = ctm.sym_norm(*ctm.qr_step(C, T, a))
    e, Cb, Tb, Asb = energy_backward(C, T, As, h, h_nnn, J2)
    n0 = np.sqrt(np.sum(Cb * Cb) + np.sum(Tb * Tb))
    ab = np.zeros_like(a)
    n_iter = None
    for it in range(0, max_iter, 2):
        for Ci, Ti in ((C1, T1), (C, T)):
            Cb, Tb, abi = qr_step_backward(Ci, Ti, a, Cb, Tb)
            ab += abi
        if np.sqrt(np.sum(Cb * Cb) + np.sum(Tb * Tb)) <= tol * n0:
            n_iter = it + 2
            break
    Asb = Asb + double_layer_backward(As, ab)
    return e, prepare_backward(A_raw, Asb), n_iter
