"""GPU parity of the J1-J2 energy and its gradient (J1-J2 paragraph).

The plaquette term 2 J2 <S.S> of a diagonal pair, and its hand-written reverse
(the four open and one closed enlarged corner, the cyclic product and their
adjoints), against the oracle's forward and reverse mode: elementwise at
small sizes (oracle run in the test), and at D = 6, chi = 72, D = 7, chi = 98
and chi = 196 against figures the oracle stored (tests/golden/, written by
tests/golden/make_qrctm_golden.py).  Tolerances: energy 1e-12 relative from
the same environment, 1e-10 after independent warm-ups; gradient 1e-9
relative (the same function, FP64 on both sides).
"""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_2505_00494_amd as P  # noqa: E402
from oracle import adjoint as adj  # noqa: E402
from oracle import ctmrg as ctm  # noqa: E402
from synth import inputs as inp  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
H1, H2, J2 = inp.heisenberg_bond_rotated(), inp.heisenberg_bond(), 0.5


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda:0")


def _env(d, D, chi, seed, steps):
    A = inp.random_site_tensor(d, D, seed)
    As = ctm.prepare_site_tensor(A)
    a = ctm.double_layer(As)
    C, T = ctm.warmup_env(a, chi, ctm.identity_boundary_vector(D))
    for _ in range(steps):
        C, T = ctm.sym_norm(*ctm.qr_step(C, T, a))
    return A, C, T


@pytest.mark.parametrize("D,chi,k,split", [(2, 16, 0, 1), (2, 16, 3, 1), (3, 27, 1, 1), (3, 27, 2, 0),
                                           (4, 32, 1, 1)])
def test_j1j2_gradient_matches_oracle(D, chi, k, split):
    print(f"j1j2 grad D={D} chi={chi} k={k} edge_split={split}", flush=True)
    A, C, T = _env(2, D, chi, seed=2, steps=6)
    e_ref, g_ref = adj.energy_grad_k(A, C, T, k, H1, H2, J2)
    ctx = P.Context(_dev(A), chi, n_warmup=0, k_tracked=k, edge_split=split)
    ctx.set_env(_dev(C), _dev(T))
    e, g = ctx.energy_grad(H1, H2, J2)
    g = g.cpu().numpy()
    assert abs(e - e_ref) < 1e-12 * abs(e_ref)
    assert np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref) < 1e-9
    # the plaquette part is really there: the nearest-neighbour gradient differs
    _, g_nn = ctx.energy_grad(H1)
    assert np.linalg.norm(g_nn.cpu().numpy() - g) > 1e-3 * np.linalg.norm(g)
    assert abs(np.sum(g * A)) < 1e-10 * np.linalg.norm(g) * np.linalg.norm(A)
    ctx.close()


def test_j1j2_gradient_matches_gpu_finite_differences():
    d, D, chi, k = 2, 2, 16, 2
    A, C, T = _env(d, D, chi, seed=4, steps=6)
    ctx = P.Context(_dev(A), chi, n_warmup=0, k_tracked=k)
    ctx.set_env(_dev(C), _dev(T))
    _, g = ctx.energy_grad(H1, H2, J2)
    g = g.cpu().numpy().ravel()

    def energy(Ax):
        ctx.set_tensor(_dev(Ax))
        ctx.set_env(_dev(C), _dev(T))
        ctx.step(k)
        return ctx.energy(H1, H2, J2)

    idx = inp.fd_entries(d, D, 4, n=8)
    fd = []
    for i in idx:
        Ap, Am = A.ravel().copy(), A.ravel().copy()
        Ap[i] += 1e-6
        Am[i] -= 1e-6
        fd.append((energy(Ap.reshape(A.shape)) - energy(Am.reshape(A.shape))) / 2e-6)
    assert np.linalg.norm(np.array(fd) - g[idx]) / np.linalg.norm(g[idx]) < 1e-6
    ctx.close()


def _oracle_fixed_point(A, D, chi):
    # an elementwise fixed point of two QR steps (the fixed-point scheme's condition)
    a = ctm.double_layer(ctm.prepare_site_tensor(A))
    r = ctm.ctmrg(a, chi, ctm.identity_boundary_vector(D), tol=1e-14, max_steps=3000)
    C, T = r.C, r.T
    for _ in range(3000):
        Cn, Tn = ctm.sym_norm(*ctm.qr_step(*ctm.sym_norm(*ctm.qr_step(C, T, a)), a))
        dd = max(np.abs(Cn - C).max(), np.abs(Tn - T).max())
        C, T = Cn, Tn
        if dd < 1e-15:
            break
    assert dd < 1e-15, "not an elementwise fixed point"
    return C, T


@pytest.mark.parametrize("D,chi,seed", [(2, 8, 3), (3, 18, 4)])
def test_j1j2_fixed_point_gradient_matches_oracle(D, chi, seed):
    A = inp.random_site_tensor(2, D, seed)
    C, T = _oracle_fixed_point(A, D, chi)
    e_ref, g_ref, n_ref = adj.energy_grad_fixed_point(A, C, T, H1, tol=1e-12, h_nnn=H2, J2=J2)
    assert n_ref is not None
    fp = P.Context(_dev(A), chi, n_warmup=0, grad_mode=P.GRAD_FIXED_POINT, fp_tol=1e-12,
                   fp_max_iter=4000)
    fp.set_env(_dev(C), _dev(T))
    e, g = fp.energy_grad(H1, H2, J2)
    assert fp.grad_converged
    assert abs(fp.stats()["grad_steps"] - n_ref) <= 2
    g = g.cpu().numpy()
    assert abs(e - e_ref) < 1e-12 * abs(e_ref)
    assert np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref) < 1e-9
    fp.close()


@pytest.mark.parametrize("name", ["j1j2_d2_D6_chi72", "j1j2_d2_D7_chi98", "j1j2_d2_D7_chi196"])
def test_j1j2_large_against_stored_oracle(name):
    path = os.path.join(GOLDEN, name + ".json")
    with open(path) as f:
        gd = json.load(f)
    d, D, chi = gd["d"], gd["D"], gd["chi"]
    print(f"{name}: warm-up", flush=True)
    A = inp.random_site_tensor(d, D, gd["seed"])
    k = gd["k_tracked"] if gd["k_tracked"] is not None else 1
    ctx = P.Context(_dev(A), chi, k_tracked=k)
    for i in range(gd["qr_steps"]):
        dl = ctx.step(1)
        e = ctx.energy(H1, H2, gd["J2"])
        print(f"step {i + 1}: delta {dl:.6e} energy {e:.15f}", flush=True)
        assert abs(e - gd["energies"][i]) < 1e-10 * abs(gd["energies"][i]), i
    if gd["k_tracked"] is not None:
        print("gradient", flush=True)
        ek, gA = ctx.energy_grad(H1, H2, gd["J2"])
        assert abs(ek - gd["energy_k"]) < 1e-10 * abs(gd["energy_k"])
        gf = gA.cpu().numpy().ravel()
        ref = np.array(gd["grad_entries"])
        got = gf[np.array(gd["grad_entries_index"])]
        assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-9
        assert abs(np.linalg.norm(gf) - gd["grad_norm"]) < 1e-9 * gd["grad_norm"]
    ctx.close()


def test_lbfgs_lowers_the_j1j2_energy():
    # the project's own minimiser (paper_2505_00494_amd.optim) on the J1-J2
    # energy: every accepted step satisfies the Armijo condition, so the energy
    # falls monotonically; the environment of each accepted step is reused
    from paper_2505_00494_amd import optim
    A0 = inp.random_site_tensor(2, 2, 6)
    ctx = P.Context(_dev(A0), 16, k_tracked=4)
    ctx.converge(1e-10, 300)
    res = optim.lbfgs(ctx, A0, H1, H2, J2, iters=6, tol=1e-10, max_steps=300)
    es = [h.energy for h in res.history]
    print("L-BFGS energies:", es, flush=True)
    assert len(es) >= 4
    assert all(b < a for a, b in zip(es, es[1:]))
    assert es[-1] < es[0]
    # the reported energy is that of the returned tensor from a fresh context
    chk = P.Context(_dev(res.A), 16)
    chk.converge(1e-10, 600)
    assert abs(chk.energy(H1, H2, J2) - res.energy) < 1e-6
    ctx.close()
    chk.close()
