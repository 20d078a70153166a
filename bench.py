#!/usr/bin/env python3
"""QR-CTMRG throughput on one MI355X: steps/s and FP64 MFMA TFLOP/s.

Workload: C4v QR-CTMRG on a random C4v-symmetrised site tensor, d = 2, D = 6,
chi = 144 (reduced corner 5184 x 144), FP64.  One "step" is one full QR-CTMRG
step: reduced corner, QR (Cholesky-QR2, Householder where it is rejected),
T' = Q^T (T a) Q, accelerated corner, symmetrise/normalise and the
corner-spectrum convergence measure.  The value is the library's default form:
FP64, with the edge contraction's middle product (3b) done by the fused
ket/bra-split kernel.

The environment is initialised (C4v average, double layer, boundary, standard
warm-up step) before the timed region; W untimed steps follow; then exactly K
steps are timed between two stream synchronisations.  Every phase is then timed
per launch with HIP events on the library's stream in a second pass; the
roofline figure is for the phase with the largest share of the step, and the
per-kernel figures for the others follow.  The CPU baseline is the FP64 oracle
on the host cores on a bounded sample of the same workload.

Also reported, at D = 6, chi = 144 and (block "target") at the largest
single-GPU case D = 8, chi = 256, same tensor seed: the forms of the step,
each with the 3b kernel the library reports for it -- the plain form (3b as
one FP64 GEMM with the double-layer tensor, 2 chi^2 D^8 flops), the FP32 form
(default split form on the FP32 matrix cores) and the split-BF16 form (plain
form, 3b as six bf16 products of split planes) -- with their speed-ups over
FP64 of the same 3b form and their energy errors against it after 20 steps
from one environment, and the time of one dE/dA (k tracked steps, energy and
the reverse pass).

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_MFMA_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0

# Sources whose change makes a stored traffic measurement stale, per kernel.
TRAFFIC_SOURCES = {
    "qr": ("paper_2505_00494_amd/csrc/qr.hip", "paper_2505_00494_amd/csrc/qr.h",
           "paper_2505_00494_amd/csrc/qr_chol.hip", "paper_2505_00494_amd/csrc/gemm.hip",
           "paper_2505_00494_amd/csrc/common.h"),
    "edge_3b": ("paper_2505_00494_amd/csrc/edge_split.hip", "paper_2505_00494_amd/csrc/edge_split.h",
                "paper_2505_00494_amd/csrc/common.h"),
    "edge_3c": ("paper_2505_00494_amd/csrc/gemm.hip", "paper_2505_00494_amd/csrc/step_gemms.h",
                "paper_2505_00494_amd/csrc/common.h"),
}


def flops_3b(chi: int, D: int) -> float:
    """3b as one GEMM with the double-layer tensor."""
    return 2.0 * chi * chi * float(D) ** 8


def kernel_figures(d, D, chi):
    """Algorithmic flops and HBM bytes per launch of each phase's kernel (FP64).

    qr: Householder R (2mn^2 - 2n^3/3) and the explicit thin Q (same again) of
    the m x n reduced corner, reading it once and writing Q (m n) and R (n^2).
    edge_3b: the fused split kernel, 4 d chi^2 D^6 flops; reads Y, writes Z.
    edge_3a / edge_3c: 2 chi^3 D^4 each; the operands once and the result once.
    """
    m, n = chi * D * D, chi
    R = D * D
    b = 8.0
    y = float(chi) * chi * R * R
    return {
        "qr": (4.0 * m * n * n - 4.0 * n ** 3 / 3.0, b * (2.0 * m * n + n * n)),
        "edge_3b": (4.0 * d * chi * chi * float(D) ** 6, b * 2.0 * y),
        "edge_3a": (2.0 * float(chi) ** 3 * R * R, b * (m * n + chi * chi * R + y)),
        "edge_3c": (2.0 * float(chi) ** 3 * R * R, b * (y + m * n + chi * chi * R)),
    }


def traffic_source_hash(kernel: str) -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in TRAFFIC_SOURCES[kernel]:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel, d, D, chi):
    """HBM bytes per launch of a phase's kernel from the committed counter summary.

    The summary (profiles/{kernel}_traffic_d{d}_D{D}_chi{chi}.md) holds the
    FETCH_SIZE and WRITE_SIZE readings per dispatch, each already scaled by
    what the same counter reads for a plain copy of known size, and the hash
    of the kernel sources they were taken with.  Returns None when there is no
    summary or the kernel has changed since.
    """
    if kernel not in TRAFFIC_SOURCES:
        return None
    path = os.path.join(ROOT, "profiles", f"{kernel}_traffic_d{d}_D{D}_chi{chi}.md")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            m = line.strip().lstrip("-* ").split(":", 1)
            if len(m) == 2:
                vals[m[0].strip()] = m[1].strip().strip("`")
    try:
        if vals["kernel_source_sha256"] != traffic_source_hash(kernel):
            return None
        return {"bytes": float(vals["fetch_bytes_per_launch"]) + float(vals["write_bytes_per_launch"]),
                "fetch_bytes": float(vals["fetch_bytes_per_launch"]),
                "write_bytes": float(vals["write_bytes_per_launch"]),
                "algorithmic_bytes": float(vals["algorithmic_bytes_per_launch"])}
    except (KeyError, ValueError):
        return None


def copy_calibration(mib: int):
    """A plain device copy of known size, for scaling the HBM byte counters."""
    import torch
    n = mib << 20
    src = torch.ones(n // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.mul(src, 1.0, out=dst)      # one elementwise kernel: reads n bytes, writes n bytes
    torch.cuda.synchronize()
    print(f"# copy calibration: 3 elementwise copies of {n} bytes", file=sys.stderr, flush=True)


def cpu_baseline(d, D, chi, seed, budget_s=20.0):
    """Oracle QR steps on the host (FP64, numpy/OpenBLAS) for about budget_s seconds."""
    from oracle import ctmrg as ctm
    from synth import inputs as inp
    try:
        from threadpoolctl import threadpool_info
        threads = max(int(i.get("num_threads", 1)) for i in threadpool_info())
    except Exception:
        threads = os.cpu_count() or 1
    A = inp.random_site_tensor(d, D, seed)
    As = ctm.prepare_site_tensor(A)
    a = ctm.double_layer(As)
    C, T = ctm.warmup_env(a, chi, ctm.identity_boundary_vector(D))
    s_prev = ctm.spectrum(C)
    n = 0
    t0 = time.perf_counter()
    while True:
        C, T = ctm.sym_norm(*ctm.qr_step(C, T, a))
        s = ctm.spectrum(C)
        ctm.spectrum_delta(s, s_prev)
        s_prev = s
        n += 1
        el = time.perf_counter() - t0
        if el > budget_s or n >= 200:
            break
    return {"value": n / el, "unit": "steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} QR-CTMRG steps (d={d}, D={D}, chi={chi}, seed {seed}) after the "
                      f"oracle's own warm-up, {el:.1f} s"}


def _timed_steps(torch, c, steps, warmup):
    if warmup:
        c.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    c.step(steps)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def _phases(c, nt):
    c.set_timing(True)
    c.step(nt)
    st = c.stats()
    c.set_timing(False)
    return {k: v / st["timed_steps"] for k, v in st["ms_phase"].items()}, st


def measure_forms(P, A, chi, C0, T0, fp64_sps, args, nt):
    """The plain form and the mixed forms from one environment (C0, T0).

    Each form: steps/s, per-phase ms, the 3b kernel the library reports, the
    speed-up over FP64 of the same 3b form (and over the default FP64 form),
    and the energy after args.acc_steps steps against as many FP64 steps of the
    same 3b form from (C0, T0)."""
    import torch
    from synth import inputs as inp
    h = inp.heisenberg_bond_rotated()
    D = int(A.shape[1])

    def one(precision, split):
        c = P.Context(A, chi, precision=precision, n_warmup=0, edge_split=split)
        c.set_env(C0, T0)
        el = _timed_steps(torch, c, args.steps, args.warmup)
        ms, st = _phases(c, nt)
        c.set_env(C0, T0)
        c.step(args.acc_steps)
        e = c.energy(h)
        r = {"steps_per_s": args.steps / el, "ms_per_step": 1e3 * el / args.steps,
             "tflops": st["flops_per_step"] * args.steps / el / 1e12, "ms_per_phase": ms,
             "edge_3b_kernel": st["edge_3b_kernel"], "energy": e}
        c.close()
        torch.cuda.empty_cache()
        return r

    plain = one(P.PREC_FP64, 0)
    plain["form"] = "FP64, 3b as one GEMM with the double-layer tensor (2 chi^2 D^8 flops)"
    t3b = flops_3b(chi, D) / (plain["ms_per_phase"]["edge_3b"] * 1e-3) / 1e12
    plain.update({"gemm_3b_tflops": t3b, "gemm_3b_frac_fp64_peak": t3b / FP64_MFMA_PEAK_TFLOPS,
                  "default_form_speedup": fp64_sps / plain["steps_per_s"]})
    split64 = one(P.PREC_FP64, 1)   # the default FP64 form again, for its energy after acc_steps
    fp32 = one(P.PREC_FP32_MFMA, 1)
    fp32["form"] = ("FP32: the default (split 3b) form with every contraction on the FP32 matrix "
                    "cores (FP32 products, FP32 sums over at most 512 of K); QR, normalisation, "
                    "spectrum FP64")
    bf16 = one(P.PREC_BF16X6_MFMA, 0)
    bf16["form"] = ("split-BF16: the plain form with 3a writing Y as three bf16 planes and 3b as six "
                    "bf16 products of planes (FP32 accumulation), the smaller products on the FP32 "
                    "matrix cores; QR, normalisation, spectrum FP64")
    for r, ref, ref_sps in ((fp32, split64, fp64_sps), (bf16, plain, plain["steps_per_s"])):
        r["speedup_vs_fp64_same_form"] = r["steps_per_s"] / ref_sps
        r["speedup_vs_fp64_default_form"] = r["steps_per_s"] / fp64_sps
        r["speedup_vs_fp64_plain_form"] = r["steps_per_s"] / plain["steps_per_s"]
        r["energy_fp64_same_form"] = ref["energy"]
        r["energy_rel_err_vs_fp64"] = abs(r["energy"] - ref["energy"]) / abs(ref["energy"])
        r["accuracy_steps"] = args.acc_steps
    return {"plain_fp64": plain, "mixed_fp32": fp32, "mixed_bf16x6": bf16,
            "mixed_speedup_headline": {
                "fp32_over_fp64_default_form": fp32["speedup_vs_fp64_same_form"],
                "bf16x6_over_fp64_plain_form": bf16["speedup_vs_fp64_same_form"],
                "fp32_over_fp64_plain_form": fp32["speedup_vs_fp64_plain_form"]}}


def measure_grad(P, A, chi, ctx, k, keep_yz):
    """One dE/dA (k tracked steps, energy, reverse pass) from ctx's environment."""
    import torch
    from synth import inputs as inp
    h = inp.heisenberg_bond_rotated()
    C0, T0 = ctx.get_env()
    g = P.Context(A, chi, n_warmup=0, k_tracked=k)
    g.set_env(C0, T0)
    g.energy_grad(h)                       # warm-up call
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e, dA = g.energy_grad(h)
    torch.cuda.synchronize()
    out = {"ms": 1e3 * (time.perf_counter() - t0), "k_tracked": k, "energy": e,
           "grad_norm": float(dA.norm()), "qr_fallbacks": g.stats()["qr_fallbacks"]}
    g.close()
    torch.cuda.empty_cache()
    if keep_yz:
        # each tracked step's Y and Z kept (2 k chi^2 D^4 doubles more workspace)
        kc = P.Context(A, chi, n_warmup=0, k_tracked=k, grad_keep_yz=1)
        kc.set_env(C0, T0)
        kc.energy_grad(h)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, dk = kc.energy_grad(h)
        torch.cuda.synchronize()
        out["ms_kept_yz"] = 1e3 * (time.perf_counter() - t0)
        out["kept_yz_rel_diff"] = float((dk - dA).norm() / dA.norm())
        kc.close()
        del dk
    del dA
    torch.cuda.empty_cache()
    return out


def measure_lbfgs(P, inp, torch, args):
    """The J1-J2 workload at d = 2, D = 7, chi = 196, J2/J1 = 0.5: ten L-BFGS
    steps of the library's own minimiser (paper_2505_00494_amd.optim) from the
    symmetrised random tensor, each energy and gradient from the fixed-point
    scheme at the converged environment (the checkpointed scheme where the
    environment is not a fixed point), the environment reused between accepted
    steps; then the energy of the final tensor in FP64 and in the mixed FP32
    form from the same environment, and their relative difference."""
    from paper_2505_00494_amd import optim
    D, chi, d, J2 = 7, 196, 2, 0.5
    h1, h2 = inp.heisenberg_bond_rotated(), inp.heisenberg_bond()
    print(f"# L-BFGS block d={d} D={D} chi={chi} J2={J2}", file=sys.stderr, flush=True)
    A0 = inp.random_site_tensor(d, D, args.seed)
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    ctx = P.Context(torch.as_tensor(A0, device=dev), chi, grad_mode=P.GRAD_FIXED_POINT)
    fb = P.Context(torch.as_tensor(A0, device=dev), chi, n_warmup=0)
    ok, steps0, dl0 = ctx.converge(args.lbfgs_tol, args.lbfgs_max_steps)

    def cb(r):
        print(f"# L-BFGS it {r.it}: E {r.energy:.12f} |g| {r.grad_norm:.3e} step {r.step:.3e} "
              f"evals {r.evals} env steps {r.env_steps} delta {r.env_delta:.2e} "
              f"scheme {r.grad_scheme} ({r.seconds:.1f} s)", file=sys.stderr, flush=True)

    res = optim.lbfgs(ctx, A0, h1, h2, J2, iters=args.lbfgs_iters, tol=args.lbfgs_tol,
                      max_steps=args.lbfgs_max_steps, fallback_ctx=fb, callback=cb)
    el = time.perf_counter() - t0
    C1, T1 = ctx.get_env()
    ctx.close()
    fb.close()
    torch.cuda.empty_cache()
    At = torch.as_tensor(np.ascontiguousarray(res.A), device=dev)
    energies = {}
    for name, prec in (("fp64", P.PREC_FP64), ("mixed_fp32", P.PREC_FP32_MFMA)):
        c = P.Context(At, chi, n_warmup=0, precision=prec)
        c.set_env(C1, T1)
        okc, st, dlc = c.converge(args.lbfgs_tol, args.lbfgs_max_steps)
        energies[name] = {"energy": c.energy(h1, h2, J2), "converged": okc, "steps": st,
                          "delta": dlc}
        c.close()
        torch.cuda.empty_cache()
    e64, e32 = energies["fp64"]["energy"], energies["mixed_fp32"]["energy"]
    return {"config": {"d": d, "D": D, "chi": chi, "J2": J2, "seed": args.seed,
                       "iters": args.lbfgs_iters, "tol": args.lbfgs_tol,
                       "max_steps": args.lbfgs_max_steps},
            "initial_env": {"converged": ok, "steps": steps0, "delta": dl0},
            "seconds": el,
            "history": [dict(r.__dict__) for r in res.history],
            "final_energy": res.energy,
            "final_energy_fp64_vs_mixed_fp32": energies,
            "mixed_energy_rel_err": abs(e32 - e64) / abs(e64)}


def measure_target(P, inp, torch, args, nt):
    """The largest single-GPU case, d = 2, D = 8, chi = 256 (same seed): the
    default FP64 form with per-kernel rooflines, the plain and mixed forms, and
    one dE/dA with k = args.k."""
    D, chi, d = 8, 256, 2
    steps, warmup = args.target_steps, 2
    print(f"# target block d={d} D={D} chi={chi}", file=sys.stderr, flush=True)
    A = torch.as_tensor(inp.random_site_tensor(d, D, args.seed), device="cuda:0")
    t0 = time.perf_counter()
    c = P.Context(A, chi)
    t_init = time.perf_counter() - t0
    el = _timed_steps(torch, c, steps, warmup)
    sps = steps / el
    ms, st = _phases(c, nt)
    figs = kernel_figures(d, D, chi)
    kern = {}
    for k, (fl, by) in figs.items():
        t = ms[k] * 1e-3
        kern[k] = {"ms_per_launch": ms[k], "achieved_tflops": fl / t / 1e12,
                   "frac_fp64_peak": fl / t / 1e12 / FP64_MFMA_PEAK_TFLOPS,
                   "algorithmic_hbm_gbs": by / t / 1e9}
    out = {"config": {"d": d, "D": D, "chi": chi, "seed": args.seed}, "steps": steps,
           "warmup": warmup, "init_s": t_init, "steps_per_s": sps, "ms_per_step": 1e3 * el / steps,
           "tflops": st["flops_per_step"] * sps / 1e12, "flops_per_step": st["flops_per_step"],
           "ms_per_phase": ms, "kernels": kern, "edge_3b_kernel": st["edge_3b_kernel"],
           "qr_fallbacks": st["qr_fallbacks"]}
    C0, T0 = c.get_env()
    sub = argparse.Namespace(steps=steps, warmup=warmup, acc_steps=args.acc_steps)
    if not args.no_mixed:
        out["forms"] = measure_forms(P, A, chi, C0, T0, sps, sub, nt)
    if not args.no_grad:
        out["grad"] = measure_grad(P, A, chi, c, args.k, keep_yz=False)
    c.close()
    del C0, T0
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--D", type=int, default=6)
    ap.add_argument("--chi", type=int, default=144)
    ap.add_argument("--d", type=int, default=2)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-grad", action="store_true")
    ap.add_argument("--no-target", action="store_true",
                    help="skip the d=2, D=8, chi=256 block")
    ap.add_argument("--target-steps", type=int, default=10)
    ap.add_argument("--acc-steps", type=int, default=20)
    ap.add_argument("--k", type=int, default=10, help="tracked steps of the gradient")
    ap.add_argument("--converge-tol", type=float, default=0.0,
                    help="time to a converged environment per form (0: skip)")
    ap.add_argument("--converge-max", type=int, default=600)
    ap.add_argument("--chi-sweep", type=str, default="",
                    help="comma-separated chi values: also time the default form at each")
    ap.add_argument("--lbfgs", action="store_true",
                    help="also run ten L-BFGS steps on the J1-J2 energy at D=7, chi=196")
    ap.add_argument("--lbfgs-iters", type=int, default=10)
    ap.add_argument("--lbfgs-tol", type=float, default=1e-10)
    ap.add_argument("--lbfgs-max-steps", type=int, default=100)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="also run a plain device copy of MIB MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this library runs on one GPU only (asked for --gpus {args.gpus}); "
              "the path would shard the 3a/3b/3c chain over the new chi index with one "
              "all-gather of T' per step", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2505_00494_amd as P
    from synth import inputs as inp

    d, D, chi = args.d, args.D, args.chi
    dev = torch.device("cuda:0")
    A = torch.as_tensor(inp.random_site_tensor(d, D, args.seed), device=dev)
    print(f"# init d={d} D={D} chi={chi}", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    ctx = P.Context(A, chi)
    t_init = time.perf_counter() - t0
    print(f"# init {t_init:.2f} s; warm-up {args.warmup} steps", file=sys.stderr, flush=True)
    if args.warmup:
        ctx.step(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    delta = ctx.step(args.steps)          # one call: K steps, one sync at the end
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    steps_per_s = args.steps / el
    st = ctx.stats()
    F = st["flops_per_step"]
    print(f"# timed {args.steps} steps in {el:.3f} s", file=sys.stderr, flush=True)

    # per-phase pass (HIP events on the library stream around every phase)
    nt = max(5, min(args.steps, 20))
    ctx.set_timing(True)
    ctx.step(nt)
    st2 = ctx.stats()
    ctx.set_timing(False)
    ms = {k: v / st2["timed_steps"] for k, v in st2["ms_phase"].items()}
    figs = kernel_figures(d, D, chi)
    names = {"qr": "QR of the reduced corner (a6): Cholesky-QR2 (Gram, Cholesky with R^-1, "
                   "product M R^-1, twice), the Householder kernel idle behind it",
             "edge_3b": "fused ket/bra-split edge contraction Z = Y (A x A) (a7 3b)",
             "edge_3a": "FP64 GEMM Y = Q^T T (a7 3a)",
             "edge_3c": "FP64 GEMM T' = Z Q (a7 3c)"}

    def roof(k):
        fl, by = figs[k]
        t = ms[k] * 1e-3
        ach = fl / t / 1e12
        tr = measured_traffic(k, d, D, chi)
        r = {"bound": "mfma", "achieved": ach, "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
             "frac": ach / FP64_MFMA_PEAK_TFLOPS, "traffic": tr["bytes"] if tr else None,
             "kernel": names[k], "phase": k, "flops_per_launch": fl, "ms_per_launch": ms[k],
             "algorithmic_bytes_per_launch": by, "algorithmic_hbm_gbs": by / t / 1e9}
        if tr:
            r["traffic_detail"] = tr
        return r

    # the phase with the largest share of the step on the library stream (the
    # spectrum runs on the auxiliary stream, overlapped with the next step)
    dom = max((k for k in figs), key=lambda k: ms[k])

    out = {
        "metric": f"QR-CTMRG steps/s (d={d}, D={D}, chi={chi}, FP64)",
        "value": steps_per_s,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * el / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"C4v QR-CTMRG step, random C4v site tensor (seed {args.seed}), "
                               f"d={d} D={D} chi={chi}", "d": d, "D": D, "chi": chi,
                   "seed": args.seed},
        "tflops": F * steps_per_s / 1e12,
        "flops_per_step": F,
        "last_delta": delta,
        "init_s": t_init,
        "ms_per_phase": ms,
        "roofline": roof(dom),
        "roofline_kernels": {k: roof(k) for k in figs},
    }
    st_default = ctx.stats()
    out["edge_3b_kernel"] = st_default["edge_3b_kernel"]
    out["qr_fallbacks"] = st_default["qr_fallbacks"]
    C0, T0 = ctx.get_env()
    if not args.no_mixed:
        out["forms"] = measure_forms(P, A, chi, C0, T0, steps_per_s, args, nt)
    if not args.no_grad:
        out["grad"] = measure_grad(P, A, chi, ctx, args.k, keep_yz=True)
    ctx.close()
    del C0, T0
    torch.cuda.empty_cache()
    if not args.no_target:
        out["target"] = measure_target(P, inp, torch, args, nt)
    if args.lbfgs:
        out["lbfgs"] = measure_lbfgs(P, inp, torch, args)
    if args.chi_sweep:
        # time per step against chi (same tensor, default form), cf. the paper's Fig. 2b
        sweep = []
        for c in [int(x) for x in args.chi_sweep.split(",") if x]:
            print(f"# chi sweep: chi={c}", file=sys.stderr, flush=True)
            sctx = P.Context(A, c)
            sctx.step(args.warmup)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sctx.step(args.steps)
            torch.cuda.synchronize()
            el_s = time.perf_counter() - t0
            sctx.set_timing(True)
            sctx.step(nt)
            sst = sctx.stats()
            sctx.close()
            torch.cuda.empty_cache()  # the next, larger chi needs its own workspace
            sps = args.steps / el_s
            sweep.append({"chi": c, "steps_per_s": sps, "ms_per_step": 1e3 * el_s / args.steps,
                          "tflops": sst["flops_per_step"] * sps / 1e12,
                          "ms_per_phase": {k: v / sst["timed_steps"]
                                           for k, v in sst["ms_phase"].items()}})
        out["chi_sweep"] = sweep
    if args.calibrate_copy:
        copy_calibration(args.calibrate_copy)
    if not args.no_cpu_baseline:
        print("# cpu baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(d, D, chi, args.seed, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
