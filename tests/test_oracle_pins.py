"""Pins of the CPU oracle against facts fixed outside it.

Each test checks the oracle against something it does not compute itself: a
number the paper prints, a textbook closed form (Onsager / Yang / the Ising
internal energy), an independent algorithm (Gram-Schmidt QR, a full explicit
contraction of a small cluster), an invariant, or central finite differences.
"""
import json
import os

import numpy as np
import pytest
from scipy import integrate, special

from oracle import adjoint as adj
from oracle import ctmrg as ctm
from oracle import observables as obs
from synth import inputs as inp

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# Closed forms (textbook, computed here, independent of the oracle).
# --------------------------------------------------------------------------


def onsager_lnz(K):
    """ln Z / N of the square-lattice Ising model (Onsager), by 2D quadrature."""
    c, s = np.cosh(2 * K), np.sinh(2 * K)
    f = lambda t1, t2: np.log(c * c - s * (np.cos(t1) + np.cos(t2)))
    v, _ = integrate.dblquad(f, 0, np.pi, 0, np.pi, epsabs=1e-14, epsrel=1e-14)
    return np.log(2.0) + v / (2.0 * np.pi ** 2)


def onsager_lnz_1d(K):
    """Same quantity from the single-integral form with kappa = 2 sinh2K / cosh^2 2K."""
    kap = 2 * np.sinh(2 * K) / np.cosh(2 * K) ** 2
    g = lambda t: np.log(0.5 * (1 + np.sqrt(1 - kap * kap * np.sin(t) ** 2)))
    v, _ = integrate.quad(g, 0, np.pi / 2, epsabs=1e-14, epsrel=1e-14, limit=200)
    return np.log(2 * np.cosh(2 * K)) + v / np.pi


def yang_magnetisation(K):
    s = np.sinh(2 * K)
    return (1 - s ** -4) ** 0.125 if s > 1 else 0.0


def ising_nn_correlation(K):
    """<s_i s_j> for nearest neighbours.

    Minus the internal energy per site (two bonds per site) is
    coth2K [1 + (2/pi)(2 tanh^2 2K - 1) K(kappa)] = 2 <s_i s_j>.
    """
    kap = 2 * np.sinh(2 * K) / np.cosh(2 * K) ** 2
    return 0.5 * (1 / np.tanh(2 * K)) * (1 + 2 / np.pi * (2 * np.tanh(2 * K) ** 2 - 1)
                                         * special.ellipk(kap * kap))


def test_closed_forms_agree():
    for K in (0.3, 0.4, 0.5):
        assert abs(onsager_lnz(K) - onsager_lnz_1d(K)) < 1e-13
    assert abs(onsager_lnz_1d(0.0) - np.log(2.0)) < 1e-15
    # d(lnZ/N)/dK = 2 <s s'> (two bonds per site)
    for K in (0.35, 0.5):
        h = 1e-5
        der = (onsager_lnz_1d(K + h) - onsager_lnz_1d(K - h)) / (2 * h)
        assert abs(der - 2 * ising_nn_correlation(K)) < 1e-8


# --------------------------------------------------------------------------
# a1: C4v average.
# --------------------------------------------------------------------------


def _projector_trace(d, D):
    n = d * D ** 4
    X = np.arange(n, dtype=np.float64).reshape(d, D, D, D, D)
    fixed = 0
    for p in ctm.c4v_leg_permutations():
        Xg = np.transpose(X, (0,) + tuple(1 + q for q in p))
        fixed += int(np.sum(Xg == X))
    return fixed / 8.0


def test_c4v_parameter_count_matches_paper():
    with open(os.path.join(GOLDEN, "c4v_parameter_count.json")) as f:
        g = json.load(f)
    assert _projector_trace(g["d"], g["D"]) == g["n"]
    for D in range(1, 9):
        assert _projector_trace(2, D) == ctm.c4v_parameter_count(2, D)


def test_c4v_projector_trace_by_basis():
    # trace of the oracle's linear map itself, applied to basis vectors
    d, D = 2, 3
    n = d * D ** 4
    tr = 0.0
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        tr += ctm.c4v_average(e.reshape(d, D, D, D, D)).ravel()[i]
    assert abs(tr - ctm.c4v_parameter_count(d, D)) < 1e-12


def test_c4v_average_is_projector_and_invariant():
    A = inp.random_site_tensor(2, 3, 7)
    P = ctm.c4v_average(A)
    assert np.abs(ctm.c4v_average(P) - P).max() < 1e-15
    for p in ctm.c4v_leg_permutations():
        assert np.abs(np.transpose(P, (0,) + tuple(1 + q for q in p)) - P).max() < 1e-15
    As = ctm.prepare_site_tensor(A)
    assert abs(np.abs(As).max() - 1.0) < 1e-15


# --------------------------------------------------------------------------
# a2/a3 + whole pipeline: classical Ising against Onsager and Yang.
# --------------------------------------------------------------------------


@pytest.mark.parametrize("variant", ["qr", "eigh"])
def test_ising_free_energy_k040(variant):
    K = 0.40
    a = inp.ising_classical_tensor(K)
    r = ctm.ctmrg(a, 32, inp.ising_boundary_vector(K), tol=1e-13, max_steps=4000,
                  variant=variant)
    assert r.converged
    assert abs(obs.ln_kappa(r.C, r.T, a) - onsager_lnz(K)) < 1e-10
    m = obs.expect_site(r.C, r.T, a, inp.ising_impurity_tensor(K))
    assert abs(m) < 1e-12


def test_ising_free_energy_infinite_temperature():
    # K = 0: every weight is 1, Z = 2^N exactly; the environment has rank 1,
    # which exercises the rank-deficient QR.
    a = inp.ising_classical_tensor(0.0)
    r = ctm.ctmrg(a, 8, inp.ising_boundary_vector(0.0), tol=1e-13, max_steps=50)
    assert abs(obs.ln_kappa(r.C, r.T, a) - np.log(2.0)) < 1e-14


def test_ising_ordered_phase_magnetisation():
    K = 0.50
    a = inp.ising_classical_tensor(K)
    r = ctm.ctmrg(a, 32, inp.ising_boundary_vector(K, biased=True), tol=1e-13,
                  max_steps=2000)
    assert abs(obs.ln_kappa(r.C, r.T, a) - onsager_lnz(K)) < 1e-10
    m = obs.expect_site(r.C, r.T, a, inp.ising_impurity_tensor(K))
    assert abs(m - yang_magnetisation(K)) < 1e-9


@pytest.mark.slow
def test_ising_near_critical_k044_improves_with_chi():
    K = 0.44
    ref = onsager_lnz(K)
    a = inp.ising_classical_tensor(K)
    errs = []
    for chi in (8, 16, 32):
        r = ctm.ctmrg(a, chi, inp.ising_boundary_vector(K), tol=1e-12, max_steps=20000)
        errs.append(abs(obs.ln_kappa(r.C, r.T, a) - ref))
    assert errs[-1] < 1e-6
    assert errs[0] > errs[1] > errs[2]


def test_double_layer_norm_network_is_ising_partition_function():
    # psi(s) = prod exp((K/2) s s') has <psi|psi> = Z(K): checks the double layer
    # (ket/bra pairing) and the bra-ket boundary initialisation.
    K = 0.40
    A = inp.ising_peps_tensor(K)
    m = np.abs(ctm.c4v_average(A)).max()
    As = ctm.prepare_site_tensor(A)
    a = ctm.double_layer(As)
    r = ctm.ctmrg(a, 32, ctm.identity_boundary_vector(2), tol=1e-13, max_steps=4000)
    lk = obs.ln_kappa(r.C, r.T, a) + 2.0 * np.log(m)
    assert abs(lk - onsager_lnz(K)) < 1e-10
    # nearest-neighbour <sz sz> of this state is the Ising correlation at K
    _, _, sz = inp.pauli()
    e = obs.energy_nn(r.C, r.T, As, np.kron(sz, sz))
    assert abs(e - 2.0 * ising_nn_correlation(K)) < 1e-9


def test_double_layer_structure():
    A = inp.random_site_tensor(2, 2, 3)
    a = ctm.double_layer(A)
    # as a (ket) x (bra) matrix the double layer is A^T A: PSD with rank <= d
    M = a.reshape(2, 2, 2, 2, 2, 2, 2, 2).transpose(0, 2, 4, 6, 1, 3, 5, 7).reshape(16, 16)
    Am = A.reshape(2, 16)
    assert np.abs(M - Am.T @ Am).max() < 1e-14
    ev = np.linalg.eigvalsh(M)
    assert ev.min() > -1e-13 and np.sum(ev > 1e-12) <= 2


# --------------------------------------------------------------------------
# a5-a9: one QR step.
# --------------------------------------------------------------------------


def _mgs_qr(M):
    """Modified Gram-Schmidt (independent of LAPACK Householder)."""
    m, n = M.shape
    Q = M.copy()
    R = np.zeros((n, n))
    for j in range(n):
        for i in range(j):
            R[i, j] = Q[:, i] @ Q[:, j]
            Q[:, j] -= R[i, j] * Q[:, i]
        R[j, j] = np.linalg.norm(Q[:, j])
        Q[:, j] /= R[j, j]
    return Q, R


def test_qr_pos_unique_factorisation():
    rng = np.random.default_rng(5)
    M = rng.standard_normal((120, 24))
    Q, R = ctm.qr_pos(M)
    assert np.abs(Q.T @ Q - np.eye(24)).max() < 1e-14
    assert np.abs(Q @ R - M).max() < 1e-13
    assert np.all(np.diag(R) >= 0) and np.abs(np.tril(R, -1)).max() == 0
    Q2, R2 = _mgs_qr(M)
    assert np.abs(Q - Q2).max() < 1e-12 and np.abs(R - R2).max() < 1e-12


def _random_env(chi, D, seed):
    rng = np.random.default_rng(seed)
    C = rng.standard_normal((chi, chi))
    T = rng.standard_normal((chi, D * D, chi))
    return ctm.sym_norm(C, T)


def test_accelerated_corner_equals_projected_enlarged_corner():
    A = ctm.prepare_site_tensor(inp.random_site_tensor(2, 2, 1))
    a = ctm.double_layer(A)
    C, T = ctm.warmup_env(a, 16, ctm.identity_boundary_vector(2))
    p = ctm.qr_step_parts(C, T, a)
    Ct = ctm.enlarged_corner(C, T, a)
    ref = p["Q"].T @ Ct @ p["Q"]
    assert np.abs(ref - p["Cp"]).max() / np.abs(ref).max() < 1e-13
    # and c~ = Q R
    assert np.abs(p["Q"] @ p["R"] - p["ct"]).max() < 1e-13


def test_step_outputs_symmetric_before_symmetrisation():
    A = ctm.prepare_site_tensor(inp.random_site_tensor(2, 2, 2))
    a = ctm.double_layer(A)
    C, T = ctm.warmup_env(a, 16, ctm.identity_boundary_vector(2))
    for step in (lambda: ctm.qr_step(C, T, a), lambda: ctm.eigh_step(C, T, a, 16)):
        Cp, Tp = step()
        assert np.abs(Cp - Cp.T).max() / np.abs(Cp).max() < 1e-13
        assert np.abs(Tp - Tp.transpose(2, 1, 0)).max() / np.abs(Tp).max() < 1e-13
    Cn, Tn = ctm.sym_norm(Cp, Tp)
    assert np.array_equal(Cn, Cn.T) and np.array_equal(Tn, Tn.transpose(2, 1, 0))


def test_warmup_count():
    assert ctm.warmup_steps_needed(2, 2, 32) == 4          # Ising 2->4->8->16->32
    assert ctm.warmup_steps_needed(4, 4, 16) == 1          # D=2, chi=16
    assert ctm.warmup_steps_needed(36, 36, 144) == 1       # D=6, chi=144
    assert ctm.warmup_steps_needed(64, 64, 256) == 1       # D=8, chi=256


# --------------------------------------------------------------------------
# a11: reduced density matrices, against explicit full-cluster contractions.
# --------------------------------------------------------------------------


def test_rdm_nn_matches_explicit_2x1_cluster():
    A = ctm.prepare_site_tensor(inp.random_site_tensor(2, 2, 11))
    C, T = _random_env(3, 2, 4)
    ao = ctm.open_double_layer(A)
    ref = np.einsum(
        "ab,aUc,cVe,ef,bLg,fRk,gh,hDi,iEj,jk,stULDM,xyVMER->stxy",
        C, T, T, C, T, T, C, T, T, C, ao, ao, optimize="greedy")
    rho = obs.rdm_nn(C, T, A)
    assert np.abs(rho - ref).max() / np.abs(ref).max() < 1e-13


def test_rdm_nnn_matches_explicit_2x2_cluster():
    A = ctm.prepare_site_tensor(inp.random_site_tensor(2, 2, 12))
    C, T = _random_env(3, 2, 5)
    ao = ctm.open_double_layer(A)
    a = ctm.double_layer(A)
    ref = np.einsum(
        "ab,aPc,cQe,ef,fRg,gSh,hi,iUj,jVk,kl,lWm,mXb,"
        "stPXIJ,QJKR,IWVL,xyKLUS->stxy",
        C, T, T, C, T, T, C, T, T, C, T, T, ao, a, a, ao, optimize="greedy")
    rho = obs.rdm_nnn(C, T, A)
    assert np.abs(rho - ref).max() / np.abs(ref).max() < 1e-12


def test_product_state_energies():
    h = inp.heisenberg_bond_rotated()
    for D in (1, 2):
        A = inp.product_state_tensor([1.0, 0.0], D)
        As = ctm.prepare_site_tensor(A)
        a = ctm.double_layer(As)
        r = ctm.ctmrg(a, 4, ctm.identity_boundary_vector(D), tol=1e-14, max_steps=20)
        # rotated Neel state: e = 2 * (-1/4)
        assert abs(obs.energy_nn(r.C, r.T, As, h) + 0.5) < 1e-14
    psi = np.array([0.6, -0.8])
    As = ctm.prepare_site_tensor(inp.product_state_tensor(psi, 2))
    a = ctm.double_layer(As)
    r = ctm.ctmrg(a, 4, ctm.identity_boundary_vector(2), tol=1e-14, max_steps=20)
    pp = np.kron(psi, psi)
    assert abs(obs.energy_nn(r.C, r.T, As, h) - 2 * pp @ h @ pp) < 1e-14


def test_eigh_and_qr_agree_on_ising_peps():
    K = 0.40
    As = ctm.prepare_site_tensor(inp.ising_peps_tensor(K))
    a = ctm.double_layer(As)
    _, _, sz = inp.pauli()
    hzz = np.kron(sz, sz)
    e = {}
    for v in ("qr", "eigh"):
        r = ctm.ctmrg(a, 16, ctm.identity_boundary_vector(2), tol=1e-13,
                      max_steps=4000, variant=v)
        e[v] = obs.energy_nn(r.C, r.T, As, hzz)
    assert abs(e["qr"] - e["eigh"]) < 1e-10


def _heisenberg_energy(D, chi, seed, variant, max_steps):
    A = inp.random_site_tensor(2, D, seed)
    As = ctm.prepare_site_tensor(A)
    a = ctm.double_layer(As)
    r = ctm.ctmrg(a, chi, ctm.identity_boundary_vector(D), tol=1e-12, max_steps=max_steps,
                  variant=variant)
    return obs.energy_nn(r.C, r.T, As, inp.heisenberg_bond_rotated()), r


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_eigh_and_qr_agree_on_heisenberg_d4_chi64(seed):
    # Heisenberg-results paragraph and Fig. 2(a): the QR scheme reaches the
    # accuracy of the eigh scheme.  Random C4v tensors, D = 4, chi = 64, the
    # rotated nearest-neighbour Heisenberg bond.  Eigh-CTMRG converges to 1e-12
    # in 22-32 steps for every seed; QR-CTMRG only for seed 4 within 400 steps
    # (seeds 1-3 end at a spectrum change of 2.8e-7, 2.0e-10 and 1.5e-5), yet
    # the energies agree to <= 6e-8 relative (measured 3.4e-10, 5.7e-9, 5.8e-8,
    # 5e-15).
    e_eigh, r_eigh = _heisenberg_energy(4, 64, seed, "eigh", 100)
    e_qr, r_qr = _heisenberg_energy(4, 64, seed, "qr", 400)
    assert r_eigh.converged
    assert abs(e_qr - e_eigh) <= 1e-6 * abs(e_eigh)
    if seed == 4:
        assert r_qr.converged and abs(e_qr - e_eigh) <= 1e-12 * abs(e_eigh)


def test_eigh_and_qr_energy_gap_shrinks_with_chi():
    # D = 2: the two truncations keep different chi-dimensional subspaces, so at
    # finite chi their converged energies differ; the difference vanishes as chi
    # grows.  Seeds 1 and 3 (short correlation length) agree at chi = 32 to
    # rounding; seed 2 (longer) differs by 9.0e-5, 1.5e-5 and 2.6e-6 at
    # chi = 16, 32 and 128 (1.2e-6 at chi = 256, measured).
    for seed in (1, 3):
        e1, r1 = _heisenberg_energy(2, 32, seed, "eigh", 200)
        e2, r2 = _heisenberg_energy(2, 32, seed, "qr", 2000)
        assert r1.converged and r2.converged
        assert abs(e1 - e2) <= 1e-12 * abs(e1)
    gap = {}
    for chi in (16, 32, 128):
        e1, r1 = _heisenberg_energy(2, chi, 2, "eigh", 200)
        e2, r2 = _heisenberg_energy(2, chi, 2, "qr", 2000)
        assert r1.converged and r2.converged
        gap[chi] = abs(e1 - e2)
    assert gap[128] < gap[32] < gap[16] and gap[128] < 5e-6


def test_corner_spectrum_and_delta_by_hand():
    # a10, written out for known eigenvalues: C = O diag(3, -1, 0.5, 0.5) O^T has
    # |eig| sorted (3, 1, 0.5, 0.5), sum 5, so s = (0.6, 0.2, 0.1, 0.1); a 2x2
    # corner with eigenvalues (-2, 2) has s = (0.5, 0.5), padded with zeros:
    # delta^2 = 0.1^2 + 0.3^2 + 0.1^2 + 0.1^2 = 0.12.
    rng = np.random.default_rng(5)
    O, _ = np.linalg.qr(rng.standard_normal((4, 4)))
    C = O @ np.diag([3.0, -1.0, 0.5, 0.5]) @ O.T
    s = ctm.spectrum(C)
    assert np.abs(s - np.array([0.6, 0.2, 0.1, 0.1])).max() < 1e-15
    O2, _ = np.linalg.qr(rng.standard_normal((2, 2)))
    s2 = ctm.spectrum(O2 @ np.diag([-2.0, 2.0]) @ O2.T)
    assert np.abs(s2 - 0.5).max() < 1e-15
    assert abs(ctm.spectrum_delta(s, s2) - np.sqrt(0.12)) < 1e-15
    assert abs(ctm.spectrum_delta(s2, s) - np.sqrt(0.12)) < 1e-15
    # invariant under scaling of C and its sign; zero change against itself
    assert np.abs(ctm.spectrum(-7.0 * C) - s).max() < 1e-15
    assert ctm.spectrum_delta(s, s) == 0.0
    # a non-symmetric input is symmetrised first: the antisymmetric part is ignored
    K = rng.standard_normal((4, 4))
    assert np.abs(ctm.spectrum(C + (K - K.T)) - s).max() < 1e-14


# --------------------------------------------------------------------------
# a12: adjoint.
# --------------------------------------------------------------------------


def test_qr_backward_matches_finite_differences():
    rng = np.random.default_rng(9)
    M = rng.standard_normal((30, 8))
    GQ = rng.standard_normal((30, 8))
    GR = np.triu(rng.standard_normal((8, 8)))
    f = lambda X: np.sum(GQ * ctm.qr_pos(X)[0]) + np.sum(GR * ctm.qr_pos(X)[1])
    Q, R = ctm.qr_pos(M)
    g = adj.qr_backward(Q, R, GQ, GR)
    fd = np.zeros_like(M)
    h = 1e-6
    for i in range(M.shape[0]):
        for j in range(M.shape[1]):
            E = np.zeros_like(M)
            E[i, j] = h
            fd[i, j] = (f(M + E) - f(M - E)) / (2 * h)
    assert np.abs(fd - g).max() / np.abs(g).max() < 1e-8


def test_regularized_triangular_inverse_by_hand():
    # 2 x 2 by hand: R = [[a, b], [0, c]], d_x = x / (x^2 + eps^2):
    # back substitution gives [[d_a, -d_a b d_c], [0, d_c]]
    a_, b_, c_ = 2.0, -0.7, 0.5
    R = np.array([[a_, b_], [0.0, c_]])
    eps_rel = 0.3
    eps = eps_rel * 2.0
    da, dc = a_ / (a_ * a_ + eps * eps), c_ / (c_ * c_ + eps * eps)
    want = np.array([[da, -da * b_ * dc], [0.0, dc]])
    assert np.abs(adj.regularized_inverse(R, eps_rel) - want).max() < 1e-15
    # a zero pivot gives a zero row and column entry instead of a division by 0
    Z = np.array([[1.0, 0.4, 0.2], [0.0, 0.0, 0.3], [0.0, 0.0, 0.5]])
    X = adj.regularized_inverse(Z, 1e-3)
    assert np.all(np.isfinite(X)) and X[1, 1] == 0.0
    # eps -> 0: the ordinary inverse (LAPACK), and a diagonal R: r / (r^2 + eps^2)
    rng = np.random.default_rng(4)
    U = np.triu(rng.standard_normal((6, 6))) + 3 * np.eye(6)
    assert np.abs(adj.regularized_inverse(U, 0.0) - np.linalg.inv(U)).max() < 1e-13
    r = np.array([1.0, -0.5, 1e-3])
    e2 = (0.1 * 1.0) ** 2
    assert np.allclose(np.diag(adj.regularized_inverse(np.diag(r), 0.1)), r / (r * r + e2),
                       rtol=1e-15, atol=0)
    # the QR adjoint with eps_rel = 0 and with a tiny eps agree
    M = rng.standard_normal((20, 6))
    Q, Rq = ctm.qr_pos(M)
    GQ, GR = rng.standard_normal((20, 6)), np.triu(rng.standard_normal((6, 6)))
    g0 = adj.qr_backward(Q, Rq, GQ, GR)
    g1 = adj.qr_backward(Q, Rq, GQ, GR, 1e-12)
    assert np.abs(g1 - g0).max() < 1e-12 * np.abs(g0).max()


def test_energy_gradient_matches_finite_differences():
    d, D, chi, k = 2, 2, 16, 4
    A = inp.random_site_tensor(d, D, 1)
    As = ctm.prepare_site_tensor(A)
    a = ctm.double_layer(As)
    r = ctm.ctmrg(a, chi, ctm.identity_boundary_vector(D), tol=1e-12, max_steps=60)
    h = inp.heisenberg_bond_rotated()
    e, g = adj.energy_grad_k(A, r.C, r.T, k, h)
    idx = inp.fd_entries(d, D, 1, n=12)
    fd = []
    for i in idx:
        Ap = A.ravel().copy()
        Am = A.ravel().copy()
        Ap[i] += 1e-6
        Am[i] -= 1e-6
        fd.append((adj.energy_k(Ap.reshape(A.shape), r.C, r.T, k, h)
                   - adj.energy_k(Am.reshape(A.shape), r.C, r.T, k, h)) / 2e-6)
    fd = np.array(fd)
    ga = g.ravel()[idx]
    assert np.linalg.norm(fd - ga) / np.linalg.norm(ga) < 1e-6
    # invariants: scale invariance and C4v symmetry of the gradient
    assert abs(np.sum(g * A)) < 1e-10 * np.linalg.norm(g) * np.linalg.norm(A)
    assert np.abs(ctm.c4v_average(g) - g).max() < 1e-14


def test_j1j2_energy_backward_matches_finite_differences():
    # J1-J2 paragraph: e = 2<h_nn> + 2 J2 <h_nnn>; the hand-written reverse of
    # the 2x2 plaquette against central differences along random directions of
    # C, T and A (the energy as a function of an arbitrary environment)
    rng = np.random.default_rng(11)
    d, D, chi = 2, 2, 6
    A = ctm.prepare_site_tensor(inp.random_site_tensor(d, D, 4))
    C = rng.standard_normal((chi, chi))
    C = C + C.T + 8 * np.eye(chi)
    T = rng.standard_normal((chi, D * D, chi))
    T = T + T.transpose(2, 1, 0)
    h1, h2, J2 = inp.heisenberg_bond_rotated(), inp.heisenberg_bond(), 0.5
    e, Cb, Tb, Ab = adj.energy_backward(C, T, A, h1, h2, J2)
    assert abs(e - obs.energy_j1j2(C, T, A, h1, h2, J2)) < 1e-14 * abs(e)
    f = lambda Cx, Tx, Ax: obs.energy_j1j2(Cx, Tx, Ax, h1, h2, J2)
    hh = 1e-6
    for _ in range(3):
        dC, dT, dA = (rng.standard_normal(x.shape) for x in (C, T, A))
        fd = (f(C + hh * dC, T + hh * dT, A + hh * dA)
              - f(C - hh * dC, T - hh * dT, A - hh * dA)) / (2 * hh)
        an = np.sum(Cb * dC) + np.sum(Tb * dT) + np.sum(Ab * dA)
        assert abs(fd - an) < 1e-7 * max(abs(an), 1e-3)
    # the next-nearest-neighbour part alone, along each argument separately
    e2, Cb2, Tb2, Ab2 = adj.energy_nnn_backward(C, T, A, h2, J2)
    g2 = lambda Cx, Tx, Ax: f(Cx, Tx, Ax) - obs.energy_nn(Cx, Tx, Ax, h1)
    for k, (bar, x) in enumerate(((Cb2, C), (Tb2, T), (Ab2, A))):
        dx = rng.standard_normal(x.shape)
        args_p = [C, T, A]
        args_m = [C, T, A]
        args_p[k] = x + hh * dx
        args_m[k] = x - hh * dx
        fd = (g2(*args_p) - g2(*args_m)) / (2 * hh)
        assert abs(fd - np.sum(bar * dx)) < 1e-7 * max(abs(fd), 1e-3), k


def test_j1j2_energy_gradient_through_tracked_steps_matches_finite_differences():
    d, D, chi, k = 2, 2, 8, 2
    A = inp.random_site_tensor(d, D, 2)
    a = ctm.double_layer(ctm.prepare_site_tensor(A))
    C, T = ctm.warmup_env(a, chi, ctm.identity_boundary_vector(D))
    for _ in range(6):
        C, T = ctm.sym_norm(*ctm.qr_step(C, T, a))
    h1, h2, J2 = inp.heisenberg_bond_rotated(), inp.heisenberg_bond(), 0.5
    e, g = adj.energy_grad_k(A, C, T, k, h1, h2, J2)
    idx = inp.fd_entries(d, D, 2, n=10)
    fd = []
    for i in idx:
        Ap = A.ravel().copy()
        Am = A.ravel().copy()
        Ap[i] += 1e-6
        Am[i] -= 1e-6
        fd.append((adj.energy_k(Ap.reshape(A.shape), C, T, k, h1, h2, J2)
                   - adj.energy_k(Am.reshape(A.shape), C, T, k, h1, h2, J2)) / 2e-6)
    fd = np.array(fd)
    ga = g.ravel()[idx]
    assert np.linalg.norm(fd - ga) / np.linalg.norm(ga) < 1e-6
    assert abs(np.sum(g * A)) < 1e-10 * np.linalg.norm(g) * np.linalg.norm(A)
    assert np.abs(ctm.c4v_average(g) - g).max() < 1e-14


def _converged_pair_env(a, chi, D, tol):
    """Environment converged under G = F o F (F one QR step + sym_norm) to max |change| < tol."""
    r = ctm.ctmrg(a, chi, ctm.identity_boundary_vector(D), tol=1e-14, max_steps=3000)
    C, T = r.C, r.T
    for _ in range(3000):
        Cn, Tn = ctm.sym_norm(*ctm.qr_step(*ctm.sym_norm(*ctm.qr_step(C, T, a)), a))
        dd = max(np.abs(Cn - C).max(), np.abs(Tn - T).max())
        C, T = Cn, Tn
        if dd < tol:
            break
    return C, T


def test_fixed_point_gradient_matches_finite_differences_of_converged_energy():
    # Discussion paragraph (fixed-point AD): dE/dA of the energy at the
    # converged environment, against central differences of that energy, each
    # side re-converged from the unperturbed fixed point
    d, D, chi, seed = 2, 2, 8, 3
    A = inp.random_site_tensor(d, D, seed)
    h = inp.heisenberg_bond_rotated()
    a = ctm.double_layer(ctm.prepare_site_tensor(A))
    C, T = _converged_pair_env(a, chi, D, 1e-15)
    e, g, n = adj.energy_grad_fixed_point(A, C, T, h, tol=1e-13)
    assert n is not None and n % 2 == 0

    def e_conv(Ap):
        Asp = ctm.prepare_site_tensor(Ap)
        ap = ctm.double_layer(Asp)
        Cc, Tc = C, T
        for _ in range(2000):
            Cn, Tn = ctm.sym_norm(*ctm.qr_step(*ctm.sym_norm(*ctm.qr_step(Cc, Tc, ap)), ap))
            dd = max(np.abs(Cn - Cc).max(), np.abs(Tn - Tc).max())
            Cc, Tc = Cn, Tn
            if dd < 1e-15:
                break
        return obs.energy_nn(Cc, Tc, Asp, h)

    idx = inp.fd_entries(d, D, seed, n=8)
    hh = 1e-5
    fd = []
    for i in idx:
        Ap = A.ravel().copy()
        Am = A.ravel().copy()
        Ap[i] += hh
        Am[i] -= hh
        fd.append((e_conv(Ap.reshape(A.shape)) - e_conv(Am.reshape(A.shape))) / (2 * hh))
    fd = np.array(fd)
    ga = g.ravel()[idx]
    assert np.linalg.norm(fd - ga) / np.linalg.norm(ga) < 1e-6
    assert abs(e - obs.energy_nn(C, T, ctm.prepare_site_tensor(A), h)) < 1e-15
    assert abs(np.sum(g * A)) < 1e-10 * np.linalg.norm(g) * np.linalg.norm(A)
    assert np.abs(ctm.c4v_average(g) - g).max() < 1e-14
    # the k-step gradient from the fixed point tends to it as k grows
    errs = [np.abs(adj.energy_grad_k(A, C, T, k, h)[1] - g).max() for k in (4, 16, 64)]
    assert errs[2] < errs[1] < errs[0] and errs[2] < 1e-8 * np.abs(g).max()
