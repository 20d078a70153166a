"""Energy minimisation of the site tensor by L-BFGS on top of the library's gradient.

The AD paragraph minimises E(A) with L-BFGS, reusing the environment of the
previous optimisation step as the starting point of the next one (but not
inside line searches).  This module is that loop, host code only: every
energy and gradient comes from ctm_converge + ctm_energy_grad (the hand-written
adjoint on the GPU); the L-BFGS two-loop recursion acts on the d*D^4 entries
of A.

* Evaluation at A: ctm_set_tensor(A), ctm_converge(tol, max_steps) from the
  current environment, then ctm_energy_grad.  The gradient scheme is the
  context's (checkpointed or fixed point); with the fixed-point scheme an
  environment that is not a fixed point of two QR steps (CTM_ESTATE, e.g.
  QR-CTMRG stalling on a random tensor) is differentiated by the checkpointed
  scheme of a second context instead, and the evaluation records that.
* Environment reuse: the environment after an accepted step is kept; every
  trial point of the next line search starts from it (ctm_set_env), so a
  rejected trial leaves nothing behind.
* Line search: backtracking from step 1 (the first iteration from 1/|g|)
  until the Armijo condition E(A + a p) <= E(A) + 1e-4 a g.p holds (at most
  max_backtracks halvings).  The curvature pair (s, y) is kept only when
  s.y > 0.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import qrctm as _q


@dataclass
class LbfgsStep:
    it: int
    energy: float
    grad_norm: float
    step: float
    evals: int
    env_steps: int
    env_delta: float
    env_converged: bool
    grad_scheme: str
    seconds: float


@dataclass
class LbfgsResult:
    A: np.ndarray
    energy: float
    history: list = field(default_factory=list)


def _flat(t):
    return t.detach().cpu().numpy().ravel().astype(np.float64)


class _Evaluator:
    """E and dE/dA at A from the contexts' environment (see the module notes)."""

    def __init__(self, ctx, h_nn, h_nnn, J2, tol, max_steps, fallback_ctx=None):
        self.ctx, self.fb = ctx, fallback_ctx
        self.h_nn, self.h_nnn, self.J2 = h_nn, h_nnn, J2
        self.tol, self.max_steps = tol, max_steps
        self.evals = 0

    def __call__(self, A):
        torch = _q._torch()
        c = self.ctx
        At = torch.as_tensor(A.reshape(c.d, c.D, c.D, c.D, c.D), dtype=torch.float64,
                             device=c.device)
        c.set_tensor(At)
        ok, steps, dl = c.converge(self.tol, self.max_steps)
        scheme = "fixed point" if c.opts.grad_mode == _q.GRAD_FIXED_POINT else "checkpointed"
        try:
            e, g = c.energy_grad(self.h_nn, self.h_nnn, self.J2)
            if scheme == "fixed point" and not c.grad_converged:
                raise _q.CTMError(_q.CTM_NOTCONV, "fixed-point series stopped early")
        except _q.CTMError as err:
            if self.fb is None or err.code not in (_q.CTM_ESTATE, _q.CTM_NOTCONV):
                raise
            Cg, Tg = c.get_env()
            self.fb.set_tensor(At)
            self.fb.set_env(Cg, Tg)
            e, g = self.fb.energy_grad(self.h_nn, self.h_nnn, self.J2)
            scheme = "checkpointed (fixed point refused: %s)" % ("not a fixed point"
                                                                 if err.code == _q.CTM_ESTATE
                                                                 else "series not converged")
        self.evals += 1
        return float(e), _flat(g), {"steps": steps, "delta": dl, "converged": ok,
                                    "scheme": scheme}


def lbfgs(ctx, A0, h_nn, h_nnn=None, J2=0.0, iters=10, history=10, tol=1e-10,
          max_steps=200, max_backtracks=20, fallback_ctx=None, callback=None):
    """Minimise the energy per site over the site tensor A by L-BFGS.

    ctx: a Context built for A0's shape (its environment is the starting one
    and is reused between accepted steps); fallback_ctx: optional Context with
    the checkpointed scheme, used where ctx's fixed-point scheme refuses the
    environment.  Returns the final A (host array), its energy and one
    LbfgsStep per iteration.
    """
    A = np.asarray(A0, dtype=np.float64).ravel().copy()
    f = _Evaluator(ctx, h_nn, h_nnn, J2, tol, max_steps, fallback_ctx)
    t0 = time.perf_counter()
    E, g, info = f(A)
    env = ctx.get_env()
    S, Y = [], []
    res = LbfgsResult(A=A.reshape(np.shape(A0)).copy(), energy=E)
    for it in range(iters):
        # two-loop recursion: p = -H g
        q = g.copy()
        alphas = []
        for s, y in reversed(list(zip(S, Y))):
            rho = 1.0 / np.dot(y, s)
            a = rho * np.dot(s, q)
            alphas.append((rho, a))
            q -= a * y
        if S:
            q *= np.dot(S[-1], Y[-1]) / np.dot(Y[-1], Y[-1])
        for (s, y), (rho, a) in zip(zip(S, Y), reversed(alphas)):
            b = rho * np.dot(y, q)
            q += (a - b) * s
        p = -q
        gp = float(np.dot(g, p))
        if not gp < 0.0:            # not a descent direction: restart from -g
            S, Y = [], []
            p = -g
            gp = float(np.dot(g, p))
        step = 1.0 if S else 1.0 / max(np.linalg.norm(g), 1e-300)
        evals0 = f.evals
        accepted = False
        for _ in range(max_backtracks + 1):
            ctx.set_env(*env)       # every trial starts from the accepted environment
            En, gn, info = f(A + step * p)
            if En <= E + 1e-4 * step * gp:
                accepted = True
                break
            step *= 0.5
        if not accepted:
            ctx.set_env(*env)
            break
        s_vec = step * p
        y_vec = gn - g
        if np.dot(s_vec, y_vec) > 1e-12 * np.linalg.norm(s_vec) * np.linalg.norm(y_vec):
            S.append(s_vec)
            Y.append(y_vec)
            if len(S) > history:
                S.pop(0)
                Y.pop(0)
        A, E, g = A + s_vec, En, gn
        env = ctx.get_env()         # reused by the next iteration
        rec = LbfgsStep(it=it + 1, energy=E, grad_norm=float(np.linalg.norm(g)), step=step,
                        evals=f.evals - evals0, env_steps=info["steps"], env_delta=info["delta"],
                        env_converged=info["converged"], grad_scheme=info["scheme"],
                        seconds=time.perf_counter() - t0)
        res.history.append(rec)
        if callback is not None:
            callback(rec)
    res.A = A.reshape(np.shape(A0))
    res.energy = E
    return res
