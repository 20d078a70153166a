#!/usr/bin/env python3
"""QR-CTMRG throughput on one MI355X: steps/s and FP64 MFMA TFLOP/s.

Workload: C4v QR-CTMRG on a random C4v-symmetrised site tensor, d = 2, D = 6,
chi = 144 (reduced corner 5184 x 144), FP64.  One "step" is one full QR-CTMRG
step: reduced corner, Householder QR, T' = Q^T (T a) Q, accelerated corner,
symmetrise/normalise and the corner-spectrum convergence measure.  The value is
the library's default form: FP64, with the edge contraction's middle product
(3b) done by the fused ket/bra-split kernel.

The environment is initialised (C4v average, double layer, boundary, standard
warm-up step) before the timed region; W untimed steps follow; then exactly K
steps are timed between two stream synchronisations.  Every phase is then timed
per launch with HIP events on the library's stream in a second pass; the
roofline figure is for the phase with the largest share of the step, and the
per-kernel figures for the others follow.  The CPU baseline is the FP64 oracle
on the host cores on a bounded sample of the same workload.

Also reported (same tensor): the plain form (3b as one GEMM with the
double-layer tensor, 2 chi^2 D^8 flops), the mixed forms (bulk contractions on
the FP32 matrix cores, or as split-BF16 products on the bf16 matrix cores) with
their speed-ups and energy errors against FP64, and the time of one dE/dA (k
tracked steps, energy and the reverse pass).

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
           "paper_2505_00494_amd/csrc/common.h"),
    "edge_3b": ("paper_2505_00494_amd/csrc/edge_split.hip", "paper_2505_00494_amd/csrc/edge_split.h",
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
    ap.add_argument("--acc-steps", type=int, default=20)
    ap.add_argument("--k", type=int, default=10, help="tracked steps of the gradient")
    ap.add_argument("--converge-tol", type=float, default=0.0,
                    help="time to a converged environment per form (0: skip)")
    ap.add_argument("--converge-max", type=int, default=600)
    ap.add_argument("--chi-sweep", type=str, default="",
                    help="comma-separated chi values: also time the default form at each")
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
    names = {"qr": "cooperative blocked Householder QR of the reduced corner (a6)",
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
    C0, T0 = ctx.get_env()
    # plain form: 3b as one FP64 GEMM with the double-layer tensor
    pctx = P.Context(A, chi, n_warmup=0, edge_split=0)
    pctx.set_env(C0, T0)
    if args.warmup:
        pctx.step(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pctx.step(args.steps)
    torch.cuda.synchronize()
    el_p = time.perf_counter() - t0
    pctx.set_timing(True)
    pctx.step(nt)
    pst = pctx.stats()
    pctx.close()
    ms_p = {k: v / pst["timed_steps"] for k, v in pst["ms_phase"].items()}
    plain_sps = args.steps / el_p
    t3b = flops_3b(chi, D) / (ms_p["edge_3b"] * 1e-3) / 1e12
    out["plain_double_layer"] = {
        "form": "FP64, 3b as one GEMM with the double-layer tensor (2 chi^2 D^8 flops)",
        "steps_per_s": plain_sps, "ms_per_step": 1e3 * el_p / args.steps,
        "tflops": pst["flops_per_step"] * plain_sps / 1e12, "ms_per_phase": ms_p,
        "gemm_3b_tflops": t3b, "gemm_3b_frac_fp64_peak": t3b / FP64_MFMA_PEAK_TFLOPS,
        "default_form_speedup": steps_per_s / plain_sps}
    # mixed forms: same tensor, bulk contractions on the FP32 matrix cores or
    # as split-BF16 products on the bf16 matrix cores; QR, normalisation and
    # spectrum in FP64
    if not args.no_mixed:
        h = inp.heisenberg_bond_rotated()
        nacc = args.acc_steps
        ctx.set_env(C0, T0)
        ctx.step(nacc)
        e64 = ctx.energy(h)
        conv_ref = {}
        for key, prec, desc in (
                ("mixed", P.PREC_FP32_MFMA,
                 "GEMMs and the fused split 3b on the fp32 matrix cores (FP32 products and "
                 "accumulation); QR, normalisation, spectrum FP64"),
                ("mixed_bf16x6", P.PREC_BF16X6_MFMA,
                 "split-BF16 form: large GEMMs as six bf16 products of three-part operands "
                 "with FP32 accumulation, the rest (the fused split 3b included) on the fp32 "
                 "matrix cores; QR, normalisation, spectrum FP64")):
            mctx = P.Context(A, chi, precision=prec, n_warmup=0)
            mctx.set_env(C0, T0)
            if args.warmup:
                mctx.step(args.warmup)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            mctx.step(args.steps)
            torch.cuda.synchronize()
            el_m = time.perf_counter() - t0
            mctx.set_timing(True)
            mctx.step(nt)
            mst = mctx.stats()
            mctx.set_timing(False)
            ms_m = {k: v / mst["timed_steps"] for k, v in mst["ms_phase"].items()}
            # accuracy: the same number of steps from the same environment,
            # energy from the FP64 energy contraction
            mctx.set_env(C0, T0)
            mctx.step(nacc)
            em = mctx.energy(h)
            conv = None
            if args.converge_tol > 0:
                # time to solution from the same environment: mixed steps down to
                # mixed_tol, then FP64 steps to the tolerance, against FP64 alone
                if "fp64" not in conv_ref:
                    ctx.set_env(C0, T0)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    ok, n, dl = ctx.converge(args.converge_tol, args.converge_max)
                    torch.cuda.synchronize()
                    conv_ref["fp64"] = {"converged": ok, "steps": n, "s": time.perf_counter() - t0,
                                        "energy": ctx.energy(h)}
                mctx.set_env(C0, T0)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ok, n, dl = mctx.converge(args.converge_tol, args.converge_max)
                torch.cuda.synchronize()
                tm = time.perf_counter() - t0
                ec = mctx.energy(h)
                r = conv_ref["fp64"]
                conv = {"tol": args.converge_tol, "converged": ok, "steps": n, "s": tm,
                        "mixed_tol": mctx.opts.mixed_tol,
                        "fp64_steps": r["steps"], "fp64_s": r["s"], "fp64_converged": r["converged"],
                        "speedup_time_to_solution": r["s"] / tm,
                        "energy_rel_err_vs_fp64": abs(ec - r["energy"]) / abs(r["energy"])}
            out[key] = {"precision": desc,
                        "steps_per_s": args.steps / el_m, "ms_per_step": 1e3 * el_m / args.steps,
                        "speedup_vs_fp64": (args.steps / el_m) / steps_per_s,
                        "speedup_vs_plain_fp64": (args.steps / el_m) / plain_sps,
                        "ms_per_phase": ms_m,
                        "energy_fp64": e64, "energy_mixed": em,
                        "energy_rel_err_vs_fp64": abs(em - e64) / abs(e64),
                        "accuracy_steps": nacc,
                        "converged_with_fp64_refinement": conv}
            mctx.close()
    # dE/dA: k tracked steps + energy + reverse pass from the current environment
    if not args.no_grad:
        gctx = P.Context(A, chi, n_warmup=0, k_tracked=args.k)
        C0, T0 = ctx.get_env()
        gctx.set_env(C0, T0)
        h = inp.heisenberg_bond_rotated()
        gctx.energy_grad(h)                       # warm-up call
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e, g = gctx.energy_grad(h)
        torch.cuda.synchronize()
        out["grad"] = {"ms": 1e3 * (time.perf_counter() - t0), "k_tracked": args.k,
                       "energy": e, "grad_norm": float(g.norm())}
        gctx.close()
        # the same with each tracked step's Y and Z kept (2 k chi^2 D^4 doubles
        # more workspace, no recomputation of 3a and 3b in the reverse sweep)
        kctx = P.Context(A, chi, n_warmup=0, k_tracked=args.k, grad_keep_yz=1)
        kctx.set_env(C0, T0)
        kctx.energy_grad(h)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ek, gk = kctx.energy_grad(h)
        torch.cuda.synchronize()
        out["grad"]["ms_kept_yz"] = 1e3 * (time.perf_counter() - t0)
        out["grad"]["kept_yz_rel_diff"] = float((gk - g).norm() / g.norm())
        kctx.close()
        del gk
        torch.cuda.empty_cache()
    ctx.close()
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
