"""Oracle forward pass: C4v CTMRG, standard (eigh) and QR variants, FP64 on the CPU.

TEST INFRASTRUCTURE ONLY (see the package docstring): never imported by the
product path.

Conventions (fixed here, shared by nothing else):
  A[s,u,l,d,r]      site tensor, legs physical / up / left / down / right.
  a[U,L,Dn,R]       double layer, U = u*D + u' (ket index major), bond D^2.
  C[x,y]            corner, chi x chi, symmetric.
  T[x,m,y]          edge: x, y boundary legs (T[x,m,y] = T[y,m,x]), m faces the bulk.
  ct[(y,m), c]      reduced corner (chi*D^2) x chi, rows (corner leg, edge inward leg).

Readings of points the paper leaves open (each also listed in the design notes):
  * the reduced corner is C.T only (QR-CTMRG paragraph: one row fewer than the
    enlarged corner, rank chi, SVD cost chi^3 D^2);
  * the QR is made unique by forcing diag(R) >= 0 (zero counts as +);
  * C and T are symmetrised and divided by their Frobenius norm after every step;
  * eigenvectors of the standard step are ordered by |lambda| descending (ties
    keep LAPACK's ascending order) and sign-fixed so that their first component
    with |v_i| >= max|v|/2 is positive;
  * convergence: s = sort(|eig C|) descending / sum, delta = ||s_k - s_{k-1}||_2
    (shorter spectra are padded with zeros).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# ----------------------------------------------------------------------------
# a1: C4v average of the site tensor (iPEPS paragraph and its parameter-count
# footnote).  The group acts on the four virtual legs in the cyclic order
# (u, l, d, r): four rotations i -> i + k and four reflections i -> k - i (mod 4).
# ----------------------------------------------------------------------------


def c4v_leg_permutations():
    perms = []
    for k in range(4):
        perms.append(tuple((i + k) % 4 for i in range(4)))
        perms.append(tuple((k - i) % 4 for i in range(4)))
    return perms


def c4v_average(A: np.ndarray) -> np.ndarray:
    """P(A) = 1/8 sum_g A o g over the 8 leg permutations of C4v."""
    out = np.zeros_like(A)
    for p in c4v_leg_permutations():
        out += np.transpose(A, (0,) + tuple(1 + q for q in p))
    return out / 8.0


def prepare_site_tensor(A_raw: np.ndarray) -> np.ndarray:
    """a1: symmetrise with P, then scale so that max |A| = 1."""
    As = c4v_average(A_raw)
    return As / np.max(np.abs(As))


def c4v_parameter_count(d: int, D: int) -> float:
    """The paper's footnote count n(D) = d/8 (D^4 + 2D^3 + 3D^2 + 2D)."""
    return d / 8.0 * (D ** 4 + 2 * D ** 3 + 3 * D ** 2 + 2 * D)


# ----------------------------------------------------------------------------
# a2: double layer (Fig. 1b): a = sum_s A (x) A, legs paired (ket, bra).
# ----------------------------------------------------------------------------


def double_layer(A: np.ndarray) -> np.ndarray:
    D = A.shape[1]
    a8 = np.einsum("sabcd,sefgh->aebfcgdh", A, A, optimize=True)
    return a8.reshape(D * D, D * D, D * D, D * D)


def open_double_layer(A: np.ndarray) -> np.ndarray:
    """a_open[s, s', U, L, Dn, R]: the double layer with the physical legs left open."""
    d, D = A.shape[0], A.shape[1]
    a8 = np.einsum("sabcd,tefgh->staebfcgdh", A, A, optimize=True)
    return a8.reshape(d, d, D * D, D * D, D * D, D * D)


def identity_boundary_vector(D: int) -> np.ndarray:
    """vec(I_D) on a paired leg (u, u'): contracts ket with bra (footnote on init)."""
    return np.eye(D).reshape(D * D)


# ----------------------------------------------------------------------------
# a3: initial boundary from the bulk tensor (footnote to the standard-CTMRG
# paragraph): contract the open boundary legs, here with a boundary vector b
# (vec(I) for a double layer, all ones for a classical weight tensor).
# ----------------------------------------------------------------------------


def init_env(a: np.ndarray, b: np.ndarray):
    C = np.einsum("U,L,ULyx->xy", b, b, a, optimize=True)
    T = np.einsum("L,xLym->xmy", b, a, optimize=True)
    return C, T


# ----------------------------------------------------------------------------
# a9: symmetrise and normalise (silent in the paper; see module docstring).
# ----------------------------------------------------------------------------


def sym_norm(C: np.ndarray, T: np.ndarray):
    Cs = 0.5 * (C + C.T)
    Ts = 0.5 * (T + T.transpose(2, 1, 0))
    return Cs / np.linalg.norm(Cs), Ts / np.linalg.norm(Ts)


# ----------------------------------------------------------------------------
# a10: corner spectrum and its change.
# ----------------------------------------------------------------------------


def spectrum(C: np.ndarray) -> np.ndarray:
    w = np.abs(np.linalg.eigvalsh(0.5 * (C + C.T)))
    w = np.sort(w)[::-1]
    return w / np.sum(w)


def spectrum_delta(s: np.ndarray, s_prev: np.ndarray) -> float:
    n = max(s.size, s_prev.size)
    x = np.zeros(n)
    y = np.zeros(n)
    x[: s.size] = s
    y[: s_prev.size] = s_prev
    return float(np.linalg.norm(x - y))


# ----------------------------------------------------------------------------
# a5: reduced corner (Fig. 1e): ct[(y,m), c] = sum_x C[y,x] T[x,m,c].
# ----------------------------------------------------------------------------


def reduced_corner(C: np.ndarray, T: np.ndarray) -> np.ndarray:
    chi, Dab, chi2 = T.shape
    return (C @ T.reshape(chi, Dab * chi2)).reshape(C.shape[0] * Dab, chi2)


# ----------------------------------------------------------------------------
# a6: unpivoted QR made unique by diag(R) >= 0.
# ----------------------------------------------------------------------------


def qr_pos(M: np.ndarray):
    Q, R = np.linalg.qr(M, mode="reduced")
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s[None, :], R * s[:, None]


# ----------------------------------------------------------------------------
# a7: edge renormalisation T' = Q^T (T a) Q (QR-CTMRG paragraph, Fig. 1c/e),
# with the enlarged edge contracted in three pairwise steps.
# ----------------------------------------------------------------------------


def renorm_edge_parts(T: np.ndarray, a: np.ndarray, Q: np.ndarray):
    chi, Dab, _ = T.shape
    chin = Q.shape[1]
    Q3 = Q.reshape(chi, Dab, chin)                       # Q3[e,u,alpha]
    Y = np.tensordot(Q3, T, axes=([0], [0]))            # [u,alpha,l,f]
    Y = Y.transpose(1, 0, 2, 3)                          # Y[alpha,u,l,f]
    Z = np.tensordot(Y, a, axes=([1, 2], [0, 1]))        # Z[alpha,f,d,r]
    Tp = np.tensordot(Z, Q3, axes=([1, 2], [0, 1]))      # Tp[alpha,r,beta]
    return Y, Z, Tp


def renorm_edge(T, a, Q):
    return renorm_edge_parts(T, a, Q)[2]


# ----------------------------------------------------------------------------
# a8: accelerated corner (Fig. 1f): C'[a,b] = sum_{g,r} T'[g,r,a] W[g,r,b],
# W[g,r,b] = sum_c R[g,c] Q[(c,r),b].  Equals Q^T Ctilde Q since ct = Q R.
# ----------------------------------------------------------------------------


def accel_corner(Tp: np.ndarray, R: np.ndarray, Q: np.ndarray) -> np.ndarray:
    chin, Dab, _ = Tp.shape
    Q3 = Q.reshape(R.shape[1], Dab, chin)
    W = np.tensordot(R, Q3, axes=([1], [0]))             # W[g,r,b]
    return np.tensordot(Tp, W, axes=([0, 1], [0, 1]))    # [a,b]


# ----------------------------------------------------------------------------
# Enlarged corner (Fig. 1d) and the standard step (standard-CTMRG paragraph).
# Ctilde[(e,dn),(c,r)] = sum T[y,l,e] a[u,l,dn,r] C[y,b] T[b,u,c].
# ----------------------------------------------------------------------------


def enlarged_corner(C, T, a):
    chi, Dab, _ = T.shape
    ct3 = reduced_corner(C, T).reshape(C.shape[0], Dab, chi)     # [y,u,c]
    G = np.tensordot(T, ct3, axes=([0], [0]))                    # [l,e,u,c]
    Ct = np.tensordot(G, a, axes=([0, 2], [1, 0]))               # [e,c,dn,r]
    Ct = Ct.transpose(0, 2, 1, 3).reshape(chi * Dab, chi * Dab)
    return 0.5 * (Ct + Ct.T)


def _sign_fix_columns(V: np.ndarray) -> np.ndarray:
    """Sign of each eigenvector: its first component with |v_i| >= max|v| / 2 is
    made positive (a rule that does not depend on which of several components
    of equal magnitude is the largest)."""
    A = np.abs(V)
    big = A >= 0.5 * A.max(axis=0, keepdims=True)
    idx = np.argmax(big, axis=0)
    s = np.sign(V[idx, np.arange(V.shape[1])])
    s[s == 0] = 1.0
    return V * s[None, :]


def eigh_step(C, T, a, chi):
    """One standard C4v CTMRG step; returns the new (C, T) before a9."""
    Ct = enlarged_corner(C, T, a)
    lam, V = np.linalg.eigh(Ct)
    order = np.argsort(-np.abs(lam), kind="stable")
    keep = order[: min(chi, lam.size)]
    U = _sign_fix_columns(V[:, keep])
    Cn = np.diag(lam[keep])
    Tn = renorm_edge(T, a, U)
    return Cn, Tn


def qr_step_parts(C, T, a):
    """One QR-CTMRG step (a5-a8); returns all intermediates, before a9."""
    ct = reduced_corner(C, T)
    Q, R = qr_pos(ct)
    Y, Z, Tp = renorm_edge_parts(T, a, Q)
    Cp = accel_corner(Tp, R, Q)
    return dict(ct=ct, Q=Q, R=R, Y=Y, Z=Z, Tp=Tp, Cp=Cp)


def qr_step(C, T, a):
    p = qr_step_parts(C, T, a)
    return p["Cp"], p["Tp"]


# ----------------------------------------------------------------------------
# Schedule: warm-up with standard steps until chi is reached (QR-CTMRG
# paragraph: 1-4 warm-up steps that also grow chi), then QR (or standard) steps
# until the corner spectrum stops changing.
# ----------------------------------------------------------------------------


def warmup_steps_needed(chi0: int, Dab: int, chi: int) -> int:
    n, c = 0, chi0
    while True:
        n += 1
        c_new = min(chi, c * Dab)
        if c_new >= chi or c_new == c:
            return n
        c = c_new


@dataclass
class CTMResult:
    C: np.ndarray
    T: np.ndarray
    steps: int
    delta: float
    deltas: list = field(default_factory=list)
    converged: bool = False


def ctmrg(a, chi, b, tol=1e-12, max_steps=200, variant="qr", n_warmup=None,
          env=None):
    """Run CTMRG on the double-layer / classical tensor a[U,L,Dn,R].

    env: optional (C, T) to start from (skips init and warm-up).
    max_steps counts the steps after the warm-up.
    """
    Dab = a.shape[0]
    if env is None:
        C, T = sym_norm(*init_env(a, b))
        nw = warmup_steps_needed(C.shape[0], Dab, chi) if n_warmup is None else n_warmup
        for _ in range(nw):
            C, T = sym_norm(*eigh_step(C, T, a, chi))
    else:
        C, T = env
    s_prev = spectrum(C)
    deltas = []
    delta = np.inf
    steps = 0
    for steps in range(1, max_steps + 1):
        if variant == "qr":
            C, T = sym_norm(*qr_step(C, T, a))
        else:
            C, T = sym_norm(*eigh_step(C, T, a, chi))
        s = spectrum(C)
        delta = spectrum_delta(s, s_prev)
        deltas.append(delta)
        s_prev = s
        if delta < tol:
            return CTMResult(C, T, steps, delta, deltas, True)
    return CTMResult(C, T, steps, delta, deltas, False)


def warmup_env(a, chi, b, n_warmup=None):
    """Init + warm-up only; the environment the QR phase starts from."""
    Dab = a.shape[0]
    C, T = sym_norm(*init_env(a, b))
    nw = warmup_steps_needed(C.shape[0], Dab, chi) if n_warmup is None else n_warmup
    for _ in range(nw):
        C, T = sym_norm(*eigh_step(C, T, a, chi))
    return C, T
