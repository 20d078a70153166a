"""GPU parity of the component kernels, called through the C ABI.

GEMM: against numpy (host BLAS, FP64) at every contraction shape family of the
step, ragged edges, transposes, alpha/beta and split-K.  QR: against the
oracle's QR (LAPACK + sign fix) elementwise, plus orthogonality and the
triangular structure, up to the full D=8 size.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_2505_00494_amd as P  # noqa: E402
from oracle import ctmrg as ctm  # noqa: E402


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda:0")


def _gemm_case(M, N, K, ta, tb, alpha, beta, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((K, M) if ta else (M, K))
    B = rng.standard_normal((N, K) if tb else (K, N))
    C0 = rng.standard_normal((M, N))
    ref = alpha * ((A.T if ta else A) @ (B.T if tb else B)) + beta * C0
    out = P.gemm(_dev(A), _dev(B), _dev(C0), trans_a=ta, trans_b=tb, alpha=alpha, beta=beta)
    got = out.cpu().numpy()
    tol = 4e-16 * K * np.abs(A).max() * np.abs(B).max() * 8 + 1e-14
    err = np.abs(got - ref).max()
    assert err < tol, (M, N, K, ta, tb, err, tol)


@pytest.mark.parametrize("M,N,K", [
    (16, 16, 4), (1, 1, 1), (17, 33, 5), (64, 64, 64), (130, 70, 19), (144, 5184, 144),
    (5184, 144, 5184), (144, 144, 5184), (300, 1296, 1296), (129, 257, 600),
])
@pytest.mark.parametrize("ta,tb", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_gemm_matches_host_blas(M, N, K, ta, tb):
    print(f"gemm M={M} N={N} K={K} ta={ta} tb={tb}", flush=True)
    _gemm_case(M, N, K, ta, tb, 1.0, 0.0, seed=M * 7 + N + K)


@pytest.mark.parametrize("ta,tb", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_gemm_vendor_sized_products_match_host_blas(ta, tb):
    # 2 M N K >= 3e10: the plain products of this size go to the vendor BLAS
    print(f"gemm (vendor size) ta={ta} tb={tb}", flush=True)
    _gemm_case(2048, 2048, 3600, ta, tb, 1.0, 0.0, seed=11 + 2 * ta + tb)
    _gemm_case(2049, 2047, 3600, ta, tb, -0.5, 0.75, seed=21 + 2 * ta + tb)


def test_gemm_alpha_beta_and_split_k():
    _gemm_case(64, 48, 20000, 1, 0, -1.5, 0.25, seed=3)   # split-K path
    _gemm_case(200, 200, 40, 0, 0, 2.0, 1.0, seed=4)


@pytest.mark.parametrize("m,n", [(64, 16), (500, 17), (1000, 37), (1024, 64), (5184, 144), (3000, 170),
                                 (9604, 196), (16384, 256), (2400, 600), (21600, 600), (4096, 1024)])
def test_qr_matches_oracle(m, n):
    print(f"qr m={m} n={n}", flush=True)
    rng = np.random.default_rng(m + n)
    M = rng.standard_normal((m, n))
    Q, R, used = P.qr(_dev(M), return_used=True)
    assert not used  # well conditioned: Cholesky-QR2
    Q, R = Q.cpu().numpy(), R.cpu().numpy()
    Qo, Ro = ctm.qr_pos(M)
    assert np.abs(np.tril(R, -1)).max() == 0.0
    assert np.all(np.diag(R) >= 0)
    assert np.abs(Q.T @ Q - np.eye(n)).max() < 1e-13
    assert np.abs(Q @ R - M).max() / np.abs(M).max() < 1e-13
    assert np.abs(Q - Qo).max() < 1e-11
    assert np.abs(R - Ro).max() / np.abs(Ro).max() < 1e-12


@pytest.mark.parametrize("m,n", [(1000, 37), (5184, 144), (16384, 256), (4096, 1024)])
def test_qr_householder_method_matches_oracle(m, n):
    print(f"qr (Householder) m={m} n={n}", flush=True)
    rng = np.random.default_rng(m + n)
    M = rng.standard_normal((m, n))
    Q, R, used = P.qr(_dev(M), method=P.QR_HOUSEHOLDER, return_used=True)
    assert used
    Q, R = Q.cpu().numpy(), R.cpu().numpy()
    Qo, Ro = ctm.qr_pos(M)
    assert np.abs(Q.T @ Q - np.eye(n)).max() < 1e-13
    assert np.abs(Q - Qo).max() < 1e-11
    assert np.abs(R - Ro).max() / np.abs(Ro).max() < 1e-12


@pytest.mark.parametrize("kappa", [1e1, 1e3, 1e7, 1e12, 1e15])
@pytest.mark.parametrize("m,n", [(5184, 144), (16384, 256)])
def test_qr_conditioning_extremes(m, n, kappa):
    # M = U diag(s) V^T with singular values spread geometrically over kappa:
    # Cholesky-QR2 takes the well-conditioned ones, the Householder kernel
    # those it rejects (kappa^2 beyond 1/u); every result is an orthonormal Q
    # with Q R = M to rounding, and Q, R differ from LAPACK's by at most about
    # kappa times the rounding unit (the condition of the thin QR factors)
    print(f"qr kappa={kappa:.0e} m={m} n={n}", flush=True)
    rng = np.random.default_rng(int(np.log10(kappa)) + n)
    U, _ = np.linalg.qr(rng.standard_normal((m, n)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    s = np.geomspace(1.0, 1.0 / kappa, n)
    M = (U * s) @ V.T
    Q, R, used = P.qr(_dev(M), return_used=True)
    if kappa <= 1e3:
        assert not used          # Cholesky-QR2 accepted it
    if kappa >= 1e12:
        assert used              # kappa^2 beyond 1/u: the Cholesky step rejects it
    Q, R = Q.cpu().numpy(), R.cpu().numpy()
    assert np.abs(np.tril(R, -1)).max() == 0.0 and np.all(np.diag(R) >= 0)
    assert np.abs(Q.T @ Q - np.eye(n)).max() < 1e-13
    assert np.abs(Q @ R - M).max() / np.abs(M).max() < 1e-13
    Qo, Ro = ctm.qr_pos(M)
    bound = 1e-14 * kappa * np.sqrt(n)
    if bound < 1e-3:
        assert np.abs(R - Ro).max() / np.abs(Ro).max() < max(bound, 1e-12)
        assert np.abs(Q - Qo).max() < max(bound, 1e-11)


def test_qr_rank_deficient_columns():
    rng = np.random.default_rng(1)
    m, n = 300, 24
    M = rng.standard_normal((m, n))
    M[:, 5] = 0.0                 # zero column
    M[:, 9] = M[:, 2]             # repeated column
    M[:, 13] = -M[:, 13] * 0.0    # another zero column (negative zero)
    Q, R, used = P.qr(_dev(M), return_used=True)
    assert used  # Cholesky-QR2 rejects it: the Householder kernel ran
    Q, R = Q.cpu().numpy(), R.cpu().numpy()
    assert np.all(np.isfinite(Q)) and np.all(np.isfinite(R))
    assert np.all(np.diag(R) >= 0)
    assert np.abs(Q.T @ Q - np.eye(n)).max() < 1e-12
    assert np.abs(Q @ R - M).max() < 1e-12
    # the independent leading columns still match the unique factorisation
    Qo, Ro = ctm.qr_pos(M[:, :5])
    assert np.abs(Q[:, :5] - Qo).max() < 1e-12
