"""GPU checks of the mixed form (bulk contractions on the FP32 matrix cores,
QR / normalisation / spectrum in FP64) against the FP64 path and the oracle.

FP32 products with FP32 accumulation carry a relative rounding of about
sqrt(K) 2^-24 per contraction; the bounds below are that budget, not the
FP64 ones.  The measured errors are reported by the benchmark.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_2505_00494_amd as P  # noqa: E402
from oracle import ctmrg as ctm  # noqa: E402
from oracle import observables as obs  # noqa: E402
from synth import inputs as inp  # noqa: E402


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda:0")


@pytest.mark.parametrize("d,D,chi", [(2, 2, 16), (2, 4, 64)])
def test_mixed_step_close_to_fp64(d, D, chi):
    A = inp.random_site_tensor(d, D, 1)
    As = ctm.prepare_site_tensor(A)
    a = ctm.double_layer(As)
    C, T = ctm.warmup_env(a, chi, ctm.identity_boundary_vector(D))
    ctx = P.Context(_dev(A), chi, n_warmup=0, precision=P.PREC_FP32_MFMA)
    ctx.set_env(_dev(C), _dev(T))
    C1, T1 = ctm.sym_norm(*ctm.qr_step(C, T, a))
    ctx.step(1)
    Cg, Tg = [x.cpu().numpy() for x in ctx.get_env()]
    # one step: FP32-class agreement elementwise, exact FP64 symmetry / norm
    assert np.abs(Cg - C1).max() / np.abs(C1).max() < 1e-4
    assert np.abs(Tg - T1).max() / np.abs(T1).max() < 1e-4
    assert np.array_equal(Cg, Cg.T)
    assert abs(np.linalg.norm(Cg) - 1.0) < 1e-14 and abs(np.linalg.norm(Tg) - 1.0) < 1e-14
    # energy after several steps from the same environment
    for _ in range(9):
        C1, T1 = ctm.sym_norm(*ctm.qr_step(C1, T1, a))
    ctx.step(9)
    h = inp.heisenberg_bond_rotated()
    e_ref = obs.energy_nn(C1, T1, As, h)
    assert abs(ctx.energy(h) - e_ref) < 1e-5 * abs(e_ref)
    ctx.close()


def test_mixed_ising_free_energy():
    from scipy import integrate
    K = 0.40
    kap = 2 * np.sinh(2 * K) / np.cosh(2 * K) ** 2
    g = lambda t: np.log(0.5 * (1 + np.sqrt(1 - kap * kap * np.sin(t) ** 2)))
    v, _ = integrate.quad(g, 0, np.pi / 2, epsabs=1e-14, epsrel=1e-14, limit=200)
    ref = np.log(2 * np.cosh(2 * K)) + v / np.pi
    a = inp.ising_classical_tensor(K)
    ctx = P.Context(a=_dev(a), bvec=_dev(inp.ising_boundary_vector(K)), chi=32,
                    precision=P.PREC_FP32_MFMA)
    ctx.converge(1e-7, 2000)
    assert abs(ctx.lnz_per_site() - ref) < 1e-6
    ctx.close()
