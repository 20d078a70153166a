"""GPU checks of the mixed forms (bulk contractions on the FP32 matrix cores,
or as six split-BF16 products on the bf16 matrix cores; QR / normalisation /
spectrum in FP64) against the FP64 path and the oracle.

FP32 products with FP32 accumulation carry a relative rounding of about
sqrt(K) 2^-24 per contraction, and the split-BF16 form keeps every term down
to 2^-24 with the same accumulation; the bounds below are that budget, not
the FP64 ones.  The measured errors are reported by the benchmark.  The
split-BF16 kernel serves products of at least 256 tiles of 128 x 128, which
first occur at D = 6, chi = 144 (3a and 3b) of the plain form (edge_split 0).
With the ket/bra-split edge contraction (edge_split 1) the split 3b runs on
the FP32 matrix cores in both mixed forms (it has no bf16 build), so the
mixed forms are checked with both settings, and ctm_stats names the 3b
kernel each one ran.
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


@pytest.mark.parametrize("split", [0, 1])
@pytest.mark.parametrize("prec,d,D,chi", [(P.PREC_FP32_MFMA, 2, 2, 16), (P.PREC_FP32_MFMA, 2, 4, 64),
                                          (P.PREC_FP32_MFMA, 2, 6, 144),
                                          (P.PREC_BF16X6_MFMA, 2, 4, 64),
                                          (P.PREC_BF16X6_MFMA, 2, 6, 144)])
def test_mixed_step_close_to_fp64(prec, d, D, chi, split):
    print(f"mixed prec={prec} d={d} D={D} chi={chi} edge_split={split}", flush=True)
    A = inp.random_site_tensor(d, D, 1)
    As = ctm.prepare_site_tensor(A)
    a = ctm.double_layer(As)
    C, T = ctm.warmup_env(a, chi, ctm.identity_boundary_vector(D))
    ctx = P.Context(_dev(A), chi, n_warmup=0, precision=prec, edge_split=split)
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


@pytest.mark.parametrize("prec", [P.PREC_FP32_MFMA, P.PREC_BF16X6_MFMA])
def test_mixed_ising_free_energy(prec):
    from scipy import integrate
    K = 0.40
    kap = 2 * np.sinh(2 * K) / np.cosh(2 * K) ** 2
    g = lambda t: np.log(0.5 * (1 + np.sqrt(1 - kap * kap * np.sin(t) ** 2)))
    v, _ = integrate.quad(g, 0, np.pi / 2, epsabs=1e-14, epsrel=1e-14, limit=200)
    ref = np.log(2 * np.cosh(2 * K)) + v / np.pi
    a = inp.ising_classical_tensor(K)
    ctx = P.Context(a=_dev(a), bvec=_dev(inp.ising_boundary_vector(K)), chi=32,
                    precision=prec)
    ctx.converge(1e-7, 2000)
    assert abs(ctx.lnz_per_site() - ref) < 1e-6
    ctx.close()


def test_split_bf16_matches_fp32_form_at_d6():
    # the split-BF16 products (3a, 3b here) against the FP32-matrix-core form
    # and FP64 over ten steps from the same environment: both mixed forms stay
    # within the FP32 budget of FP64, and of each other
    d, D, chi = 2, 6, 144
    A = inp.random_site_tensor(d, D, 1)
    ctx = P.Context(_dev(A), chi)
    C0, T0 = ctx.get_env()
    h = inp.heisenberg_bond_rotated()
    es = {}
    for prec in (P.PREC_FP64, P.PREC_FP32_MFMA, P.PREC_BF16X6_MFMA):
        c = P.Context(_dev(A), chi, n_warmup=0, precision=prec, edge_split=0)
        c.set_env(C0, T0)
        c.step(10)
        es[prec] = c.energy(h)
        c.close()
    e64 = es[P.PREC_FP64]
    print({k: abs(v - e64) / abs(e64) for k, v in es.items()}, flush=True)
    assert abs(es[P.PREC_FP32_MFMA] - e64) < 1e-5 * abs(e64)
    assert abs(es[P.PREC_BF16X6_MFMA] - e64) < 1e-5 * abs(e64)
    ctx.close()


@pytest.mark.parametrize("prec", [P.PREC_FP32_MFMA, P.PREC_BF16X6_MFMA])
def test_mixed_converge_refines_to_fp64_fixed_point(prec):
    # mixed steps down to mixed_tol, then FP64 steps: the environment that
    # ctm_converge returns is a fixed point of the FP64 iteration (further FP64
    # steps leave its energy unchanged), while the purely mixed iteration
    # stalls at the FP32 level.  (A random tensor can have several fixed points
    # at finite chi, so its energy is not compared with an FP64 run from the
    # warm-up; the benchmark reports that difference.)
    d, D, chi = 2, 4, 64
    A = inp.random_site_tensor(d, D, 3)
    h = inp.heisenberg_bond_rotated()
    ctx = P.Context(_dev(A), chi, precision=prec)
    ok, n, dl = ctx.converge(1e-11, 3000)
    assert ok and dl < 1e-11
    em = ctx.energy(h)
    C, T = ctx.get_env()
    ref = P.Context(_dev(A), chi, n_warmup=0)
    ref.set_env(C, T)
    ref.step(20)
    e64 = ref.energy(h)
    print(f"prec {prec}: {n} steps; energy change over 20 more FP64 steps "
          f"{abs(em - e64) / abs(e64):.2e}", flush=True)
    assert abs(em - e64) < 1e-10 * abs(e64)
    ref.close()
    ctx.close()


@pytest.mark.parametrize("D,chi", [(1, 4), (3, 18), (5, 50), (7, 49), (8, 64)])
def test_fp32_split_3b_close_to_fp64_split(D, chi):
    """The FP32 build of the fused split 3b at the bond dimensions whose batch
    and wave layouts the tests above do not reach: one step of the FP32 form
    against one FP64 step from the same random environment (the FP64 split
    path is checked against the oracle in test_gpu_ctm)."""
    print(f"fp32 split 3b D={D} chi={chi}", flush=True)
    rng = np.random.default_rng(100 + D)
    A = inp.random_site_tensor(2, D, 7)
    C = rng.standard_normal((chi, chi))
    C = 0.5 * (C + C.T)
    T = rng.standard_normal((chi, D * D, chi))
    T = 0.5 * (T + T.transpose(2, 1, 0))
    out = []
    for prec in (P.PREC_FP64, P.PREC_FP32_MFMA):
        ctx = P.Context(_dev(A), chi, n_warmup=0, precision=prec, edge_split=1)
        ctx.set_env(_dev(C), _dev(T))
        ctx.step(1)
        out.append([x.cpu().numpy() for x in ctx.get_env()])
        ctx.close()
    (C64, T64), (C32, T32) = out
    assert np.abs(C32 - C64).max() / np.abs(C64).max() < 1e-4
    assert np.abs(T32 - T64).max() / np.abs(T64).max() < 1e-4
    # not the FP64 result: the FP32 products did run
    assert np.abs(T32 - T64).max() > 0.0


@pytest.mark.parametrize("D,chi", [(6, 144), (8, 256)])
def test_mixed_energy_error_within_1e7(D, chi):
    # the mixed forms' energy after 20 steps against 20 FP64 steps of the same
    # 3b form from the same environment (FP32 block sums over at most 512 of K,
    # longer contractions split with FP64 partial sums): within 1e-7 relative.
    # FP32: the default form (split 3b); split-BF16: the plain form, whose 3b
    # is the bf16 product of planes
    A = torch.as_tensor(inp.random_site_tensor(2, D, 1), device="cuda:0")
    h = inp.heisenberg_bond_rotated()
    ctx = P.Context(A, chi)
    ctx.step(10)
    C0, T0 = ctx.get_env()
    for prec, split, kernel in ((P.PREC_FP32_MFMA, 1, "fused ket/bra split, FP32 matrix cores"),
                                (P.PREC_BF16X6_MFMA, 0, "double-layer GEMM as six bf16 products")):
        ref = P.Context(A, chi, n_warmup=0, edge_split=split)
        ref.set_env(C0, T0)
        ref.step(20)
        e64 = ref.energy(h)
        ref.close()
        m = P.Context(A, chi, precision=prec, n_warmup=0, edge_split=split)
        m.set_env(C0, T0)
        m.step(20)
        em = m.energy(h)
        assert m.stats()["edge_3b_kernel"].startswith(kernel)
        print(f"D={D} chi={chi} prec={prec} edge_split={split}: energy error "
              f"{abs(em - e64) / abs(e64):.2e}", flush=True)
        assert abs(em - e64) < 1e-7 * abs(e64)
        m.close()
    ctx.close()


def test_stats_name_the_3b_kernel():
    A = _dev(inp.random_site_tensor(2, 4, 1))
    want = {(P.PREC_FP64, 1): "fused ket/bra split, FP64",
            (P.PREC_FP64, 0): "double-layer GEMM, FP64",
            (P.PREC_FP32_MFMA, 1): "fused ket/bra split, FP32 matrix cores",
            (P.PREC_FP32_MFMA, 0): "double-layer GEMM, FP32 matrix cores",
            (P.PREC_BF16X6_MFMA, 1): "fused ket/bra split, FP32 matrix cores",
            (P.PREC_BF16X6_MFMA, 0): "double-layer GEMM as six bf16 products"}
    for (prec, split), name in want.items():
        c = P.Context(A, 64, precision=prec, edge_split=split)
        assert c.stats()["edge_3b_kernel"].startswith(name), (prec, split)
        c.close()
