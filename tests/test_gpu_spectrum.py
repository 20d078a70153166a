"""GPU parity of the corner spectrum (a10) and of the step schedule around it.

* The spectrum of a corner set with ctm_set_env against the oracle's sorted,
  normalised |eigvalsh|, at sizes on both sides of every storage and work-split
  boundary of the kernel (packed triangle in LDS up to 176, global rows beyond;
  eigenvalues shared by 8, 4, 2 or 1 lanes up to 64, 128, 256, 1024; column
  parts in registers up to 512, in LDS beyond), and for
  matrices with repeated eigenvalues, zero columns (a reflection that is the
  identity), a zero block and negative eigenvalues.
* QR steps where the QR's cooperative grid covers nearly every CU (d=2, D=4,
  chi=464: 232 workgroups), so each step's spectrum is queued after the next
  step's QR: environments, spectra and changes after ctm_step and after
  ctm_converge (which queues a step before reading the previous change)
  against the oracle.
Tolerance 1e-12 absolute on normalised spectra (FP64 rounding of a
tridiagonalisation and bisection to 4 eps |T|), 1e-12 relative on single steps.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_2505_00494_amd as P  # noqa: E402
from oracle import ctmrg as ctm  # noqa: E402
from synth import inputs as inp  # noqa: E402


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda:0")


def _sym_edge(rng, chi, Dab):
    T = rng.standard_normal((chi, Dab, chi))
    return 0.5 * (T + T.transpose(2, 1, 0))


def _corners(rng):
    out = []
    for n in [1, 2, 3, 17, 63, 64, 65, 128, 129, 176, 177, 255, 256, 257, 400, 512, 513, 600,
              1024]:
        out.append((f"random{n}", rng.standard_normal((n, n))))
    out.append(("identity9", np.eye(9)))
    z = rng.standard_normal((40, 40))
    z[:, 7] = 0.0
    z[7, :] = 0.0
    z[:, 30] = 0.0
    z[30, :] = 0.0
    out.append(("zero_columns40", z))
    blk = np.zeros((200, 200))
    blk[:60, :60] = rng.standard_normal((60, 60))
    out.append(("zero_block200", blk))
    q, _ = np.linalg.qr(rng.standard_normal((150, 150)))
    out.append(("signed_repeated150", (q * np.repeat([2.0, -2.0, 0.5], 50)) @ q.T))
    return out


def test_spectrum_matches_eigvalsh_at_every_size():
    rng = np.random.default_rng(11)
    A = inp.random_site_tensor(2, 1, 3)  # D = 1: Dab = 1, so any chi <= 1024 is allowed
    ctx = P.Context(_dev(A), 1024, n_warmup=0)
    for name, C in _corners(rng):
        n = C.shape[0]
        print(f"spectrum {name} n={n}", flush=True)
        ctx.set_env(_dev(C), _dev(_sym_edge(rng, n, 1)))
        s = ctx.spectrum()
        ref = ctm.spectrum(C)
        assert s.size == n
        assert np.abs(s - ref).max() < 1e-12, (name, np.abs(s - ref).max())
    ctx.close()


@pytest.fixture(scope="module")
def deferred_case():
    """Oracle reference for three QR steps at d=2, D=4, chi=464 from a random environment."""
    d, D, chi, nsteps = 2, 4, 464, 3
    rng = np.random.default_rng(5)
    A = inp.random_site_tensor(d, D, 2)
    a = ctm.double_layer(ctm.prepare_site_tensor(A))
    C0 = rng.standard_normal((chi, chi))
    C0, T0 = ctm.sym_norm(0.5 * (C0 + C0.T), _sym_edge(rng, chi, D * D))
    C, T = C0, T0
    s_prev = ctm.spectrum(C)
    dls = []
    for _ in range(nsteps):
        C, T = ctm.sym_norm(*ctm.qr_step(C, T, a))
        s = ctm.spectrum(C)
        dls.append(ctm.spectrum_delta(s, s_prev))
        s_prev = s
    return dict(A=A, chi=chi, nsteps=nsteps, C0=C0, T0=T0, C=C, T=T, s=s_prev, dls=dls)


@pytest.mark.parametrize("mode", ["step", "converge"])
def test_spectrum_queued_after_next_qr_matches_oracle(deferred_case, mode):
    r = deferred_case
    nsteps, dls = r["nsteps"], r["dls"]
    print(f"deferred spectrum schedule mode={mode} d=2 D=4 chi={r['chi']}", flush=True)
    ctx = P.Context(_dev(r["A"]), r["chi"], n_warmup=0)
    ctx.set_env(_dev(r["C0"]), _dev(r["T0"]))
    if mode == "step":
        for i in range(nsteps):
            dl = ctx.step(1)
            assert abs(dl - dls[i]) < 1e-12 + 1e-9 * dls[i], (i, dl, dls[i])
    else:
        # a tolerance no step reaches: all steps taken, the last one's change reported
        ok, taken, dl = ctx.converge(1e-300, nsteps)
        assert taken == nsteps and not ok
        assert abs(dl - dls[-1]) < 1e-12 + 1e-9 * dls[-1]
    Cg, Tg = [x.cpu().numpy() for x in ctx.get_env()]
    rel = lambda x, y: np.abs(x - y).max() / np.abs(y).max()
    assert rel(Cg, r["C"]) < 1e-10, rel(Cg, r["C"])
    assert rel(Tg, r["T"]) < 1e-10, rel(Tg, r["T"])
    assert np.abs(ctx.spectrum() - r["s"]).max() < 1e-12
    ctx.close()
