"""Throughput of the split-CTMRG hot path on one MI355X.

One step = one energy + gradient evaluation at the headline workload (2x2
unit cell of four distinct real tensors, p = 2, D = 8, chi_E = chi_I = 128,
BF16x3 contractions with FP32 accumulation, FP64 projectors): `--grad-sweeps`
split-CTMRG sweeps from a start environment (`--pre-sweeps` sweeps from the
identity boundary, the same for every timed step) with
checkpoints every `--ckpt` sweeps, the nearest-neighbour Heisenberg energy,
and dE/dA by the hand-written reverse pass.  Forward-only sweeps/s is timed
separately on the same context.  Inputs are seeded synthetic tensors already
resident in HBM.

Prints one JSON line (see the keys below); `roofline` is taken from the
library's own HIP-event timing of the dominant kernel class over the timed
steps (events on every `--timing-stride`-th launch of each class, so that the
events' host cost stays out of the timed run), `cpu_baseline` from the FP64 CPU oracle on a bounded sample (one column of
one left move at the same sizes, forward and reverse).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

WORKLOAD = "cell2x2_d2_D8_chi128_grad"
METRIC = "split-CTMRG sweeps/s + energy-grad evals/s at D=8,χ=128; MFMA fraction"

# Published MI355X peaks: dense MFMA (TFLOP/s) and HBM3E bandwidth.  A BF16x3
# product issues three BF16 MFMA products per FP32-class product, so its
# algorithmic peak is a third of the BF16 one.
HBM_PEAK_GBS = 8000.0
MFMA_PEAKS = {
    "gemm_fp64": (78.6, "fp64 MFMA"),
    "gemm_fp32": (157.3, "fp32 MFMA"),
    "gemm_bf16x3": (2500.0 / 3.0, "bf16 MFMA 2500 / 3 products"),
    "gemm_bf16x6": (2500.0 / 6.0, "bf16 MFMA 2500 / 6 products"),
    "jacobi_pair": (78.6, "fp64 MFMA"),
    "jacobi_rotate": (78.6, "fp64 MFMA"),
}


def roofline_of(name: str, ms: float, launches: float, flops: float, nbytes: float) -> dict:
    """Roofline entry of one kernel class: the bound is the one its arithmetic
    intensity (algorithmic flops per algorithmic byte) puts it under."""
    peak_tf, basis = MFMA_PEAKS[name]
    ridge = peak_tf * 1e12 / (HBM_PEAK_GBS * 1e9)
    t = ms * 1e-3
    if nbytes > 0 and (flops / nbytes) < ridge:
        achieved = nbytes / t / 1e9 if t > 0 else 0.0
        return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "peak_basis": "HBM3E"}
    achieved = flops / t / 1e12 if t > 0 else 0.0
    return {"bound": "mfma", "achieved": achieved, "peak": peak_tf, "unit": "TFLOP/s",
            "frac": achieved / peak_tf, "peak_basis": basis}


def say(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--grad-sweeps", type=int, default=4)
    ap.add_argument("--ckpt", type=int, default=4)
    ap.add_argument("--pre-sweeps", type=int, default=8,
                    help="untimed sweeps from the identity boundary that build the start environment (its corner-spectrum change is reported as start_env_delta)")
    ap.add_argument("--fwd-sweeps", type=int, default=4, help="timed forward-only sweeps for sweeps/s")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--timing-stride", type=int, default=16,
                    help="HIP events on every k-th launch of each kernel class in the timed steps")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 1 GiB device to device once (calibrates the HBM byte counters) and exit")
    ap.add_argument("--scaling", type=str, default="",
                    help="comma-separated bulk bond dimensions D: instead of the bench line, time sweeps of a 1x1 "
                         "cell at fixed chi_E = chi_I for each D and fit time ~ D^a over D >= 6 (one JSON line)")
    ap.add_argument("--scaling-chi", type=int, default=170)
    ap.add_argument("--scaling-p", type=int, default=2)
    ap.add_argument("--scaling-prec", default="bf16x3")
    ap.add_argument("--alt-yr", action="store_true",
                    help="the alternative yellow / red projectors of App. B (physical leg cut by yellow) instead "
                         "of those of App. A")
    ap.add_argument("--half-teal", action="store_true",
                    help="the teal half projectors of App. B (left halves of the patch) instead of the full ones")
    ap.add_argument("--prec", default=None, help="contraction precision of the timed steps (default: the workload's)")
    ap.add_argument("--legs", default="fp64,bf16x3,bf16x6",
                    help="other contraction precisions timed beside the headline on the same start environment "
                         "(comma-separated; the FP64 leg is the reference of the error columns); empty: none")
    ap.add_argument("--leg-steps", type=int, default=2, help="timed steps of each leg (after one warmup step)")
    ap.add_argument("--lbfgs", type=int, default=0,
                    help="instead of the bench line: this many L-BFGS iterations at the headline workload (one JSON "
                         "line with the energies and seconds per optimisation step)")
    return ap.parse_args()


# HBM traffic of the dominant kernel class, from rocprofv3 --pmc FETCH_SIZE and
# WRITE_SIZE runs of this script (scaled by the counters' reading for a copy of
# known size); valid only while the kernel's source is the one measured.
TRAFFIC_DIR = os.path.join(ROOT, "profiles")
KERNEL_SOURCE = {"jacobi_rotate": "paper_2502_10298_amd/csrc/svd.hip",
                 "jacobi_pair": "paper_2502_10298_amd/csrc/svd.hip"}


def measured_traffic(kernel: str):
    import hashlib
    path = os.path.join(TRAFFIC_DIR, f"traffic_{kernel}_{WORKLOAD}.txt")
    if kernel not in KERNEL_SOURCE or not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    src = open(os.path.join(ROOT, KERNEL_SOURCE[kernel]), "rb").read()
    if fields.get("source_sha256") != hashlib.sha256(src).hexdigest():
        return None
    try:
        return float(fields["fetch_bytes_per_launch"]) + float(fields["write_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(threads: int, n_sweeps: int) -> dict:
    """The FP64 oracle on one column of one left move at D = 8, chi = 128:
    the forward pass (projectors of every colour, the new C1, T4k, T4b, C4 of
    both rows) and its reverse pass by autograd from a seeded cotangent on the
    new tensors.  Scaled to energy-gradient evaluations per second: an
    evaluation is n_sweeps sweeps of 4 moves x Ly columns, forward and reverse
    (the energy term and its reverse pass are left out, which flatters the
    CPU)."""
    import torch
    from oracle import split_ctmrg as sc
    from paper_2502_10298_amd import inputs as inp

    if threads > 0:
        torch.set_num_threads(threads)
    used = torch.get_num_threads()
    w = inp.WORKLOADS[WORKLOAD]
    env = sc.env_from_numpy(inp.random_env(7, w["Lx"], w["Ly"], w["D"], w["chi"], w["chi"]))
    A = sc.peps_from_numpy(inp.workload_peps(WORKLOAD))
    for e in env.values():
        for k in list(e):
            e[k] = e[k].detach().requires_grad_(True)
    for k in A:
        A[k] = A[k].detach().requires_grad_(True)
    t0 = time.perf_counter()
    sc.left_move_column(env, A, w["Lx"], w["Ly"], 0, w["chi"], w["chi"])
    t1 = time.perf_counter()
    gen = torch.Generator().manual_seed(3)
    new = [t for e in env.values() for t in e.values() if t.grad_fn is not None]
    loss = sum((t * torch.randn(t.shape, generator=gen, dtype=t.dtype)).sum() for t in new)
    t2 = time.perf_counter()
    loss.backward()
    t3 = time.perf_counter()
    dt = (t1 - t0) + (t3 - t2)
    scale = n_sweeps * 4 * w["Ly"]
    return {"value": 1.0 / (dt * scale), "unit": "energy-grad evals/s", "cores": used, "kind": "oracle",
            "sample": f"one column of one left move (2 site-moves) at 2x2, D=8, chi=128, FP64, forward "
                      f"{t1 - t0:.1f} s + reverse {t3 - t2:.1f} s, scaled x{scale} to one evaluation of "
                      f"{n_sweeps} sweeps (energy term not counted)"}


def projectors_label(args) -> str:
    parts = []
    if args.alt_yr:
        parts.append("App. B alternative yellow/red")
    if args.half_teal:
        parts.append("App. B teal half projectors")
    return ", ".join(parts) if parts else "App. A"


def scaling(args) -> None:
    """Time of one sweep (four directional moves, each absorbing the ket and
    bra layers of every column) against the bulk bond dimension D at fixed
    chi_E = chi_I, on seeded Gaussian 1x1 states.  Two untimed sweeps grow the
    environment from the identity boundary to its full dimension first."""
    import numpy as np
    import torch
    from paper_2502_10298_amd import binding as b
    from paper_2502_10298_amd import inputs as inp
    chi, p = args.scaling_chi, args.scaling_p
    rows = []
    for D in [int(x) for x in args.scaling.split(",") if x]:
        A = torch.tensor(inp.peps_gaussian(700 + D, 1, 1, p, D), device="cuda:0")
        obj = b.SplitCTM(A, chi, chi, prec=args.scaling_prec, alt_yr=args.alt_yr, half_teal=args.half_teal)
        obj.sweep(2)
        torch.cuda.synchronize()
        n = 2
        t0 = time.perf_counter()
        obj.sweep(n)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / n
        rows.append({"D": D, "s_per_sweep": dt, "s_per_move": dt / 4, "jacobi_sweeps_per_call": obj.stats()[1] / n})
        say(f"D={D}: {dt:.3f} s per sweep")
        obj.close()
        del obj, A
        torch.cuda.empty_cache()
    pts = [(r["D"], r["s_per_sweep"]) for r in rows if r["D"] >= 6]
    fit = None
    if len(pts) >= 2:
        x = np.log([d for d, _ in pts])
        y = np.log([t for _, t in pts])
        fit = float(np.polyfit(x, y, 1)[0])
    print(json.dumps({"scaling": rows, "chi_E": chi, "chi_I": chi, "p": p, "cell": "1x1",
                      "prec": args.scaling_prec, "state": "seeded Gaussian", "exponent_fit_D_ge_6": fit,
                      "projectors": projectors_label(args)}),
          flush=True)


def lbfgs_run(args) -> None:
    """L-BFGS iterations of the headline workload (energy + gradient per
    evaluation, warm-started environments): energies and seconds per step."""
    import torch
    from paper_2502_10298_amd import inputs as inp
    from paper_2502_10298_amd import optimize

    w = inp.WORKLOADS[WORKLOAD]
    A0 = torch.tensor(inp.workload_peps(WORKLOAD), device="cuda:0")
    prec = args.prec or w["prec"]
    t0 = time.perf_counter()
    _, hist = optimize.lbfgs(A0, inp.workload_h(WORKLOAD), w["chi"], args.lbfgs, n_sweeps=args.grad_sweeps,
                             ckpt_every=args.ckpt, prec=prec, pre_sweeps=args.pre_sweeps, alt_yr=args.alt_yr,
                             half_teal=args.half_teal,
                             on_eval=lambda r: say(f"L-BFGS evaluation: E = {r['energy']:.10f}, "
                                                   f"{r['seconds']:.2f} s"))
    total = time.perf_counter() - t0
    iters = max(r["iteration"] for r in hist)
    print(json.dumps({"lbfgs_iterations": iters, "evaluations": len(hist), "energies": [r["energy"] for r in hist],
                      "seconds_per_evaluation": [r["seconds"] for r in hist],
                      "seconds_per_iteration": sum(r["seconds"] for r in hist) / max(iters, 1),
                      "total_seconds_with_start_environment": total, "dtype": prec,
                      "config": {"workload": WORKLOAD, "sweeps_per_eval": args.grad_sweeps, "ckpt_every": args.ckpt,
                                 "pre_sweeps": args.pre_sweeps, "projectors": projectors_label(args)}}), flush=True)


def time_steps(obj, h, args, steps):
    """`steps` energy + gradient evaluations from the context's start
    environment; returns (E, dE/dA, seconds)."""
    import torch
    e = dA = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        e, dA = obj.energy_grad(h, args.grad_sweeps, args.ckpt)
        say(f"{obj.prec_name} timed step {i} done")
    torch.cuda.synchronize()
    return e, dA, time.perf_counter() - t0


def time_sweeps(obj, flat, n):
    """Forward-only sweeps/s from the environment `flat`."""
    import torch
    obj.env_import(flat)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    obj.sweep(n)
    torch.cuda.synchronize()
    return n / (time.perf_counter() - t0)


def contraction_mfma(timing: dict, prec: str) -> dict:
    """MFMA figure of the contraction GEMMs of precision `prec`: their
    algorithmic flops (2 M N K per product) over their kernel time, against
    the dense peak of the products they issue."""
    key = {"fp64": "gemm_fp64", "fp32": "gemm_fp32", "bf16x3": "gemm_bf16x3", "bf16x6": "gemm_bf16x6"}[prec]
    ms, launches, flops, nbytes = timing[key]
    peak, basis = MFMA_PEAKS[key]
    tf = flops / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
    out = {"kernel": key, "achieved": tf, "peak": peak, "unit": "TFLOP/s", "frac": tf / peak, "peak_basis": basis,
           "ms": ms, "launches": int(launches),
           "arith_intensity_flop_per_byte": flops / nbytes if nbytes else None}
    # every GEMM class of the timed steps on the same footing (the FP64 class
    # holds the projector products, the QR block updates and the SVD lifts)
    per = {}
    for k, (cms, cl, cfl, _) in timing.items():
        if k.startswith("gemm_") and cl > 0 and cms > 0:
            pk, pb = MFMA_PEAKS[k]
            ctf = cfl / (cms * 1e-3) / 1e12
            per[k] = {"achieved": ctf, "peak": pk, "frac": ctf / pk, "ms": cms, "launches": int(cl)}
    out["classes"] = per
    if out["frac"] < 0.5:
        out["note"] = ("below 0.5 of the MFMA peak: most products are short (K <= 128) or have few output tiles, "
                       "bound by launch and load latency rather than by the matrix cores")
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (--gpus {args.gpus} requested): the split-CTMRG path "
              "runs on a single MI355X; see the sharding notes in the design document.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2502_10298_amd import binding as b
    from paper_2502_10298_amd import inputs as inp

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.scaling:
        scaling(args)
        return
    if args.lbfgs:
        lbfgs_run(args)
        return
    if args.copy_probe:
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": x.numel() * 4}), flush=True)
        return
    w = inp.WORKLOADS[WORKLOAD]
    chi = w["chi"]
    prec = args.prec or w["prec"]
    dev = torch.device("cuda:0")
    A = torch.tensor(inp.workload_peps(WORKLOAD), device=dev)
    h = inp.workload_h(WORKLOAD)

    def context(p):
        o = b.SplitCTM(A, chi, chi, prec=p, with_grad=True, n_sweeps=args.grad_sweeps, ckpt_every=args.ckpt,
                       alt_yr=args.alt_yr, half_teal=args.half_teal)
        o.prec_name = p
        return o

    obj = context(prec)
    # untimed: the start environment, grown from the identity boundary (an
    # optimisation step starts from the previous step's environment, not from
    # the boundary); every timed step and every leg starts from this same
    # environment.  It is not converged (the change of the corner spectra over
    # its last sweep is reported)
    st, n, delta = obj.sweep(args.pre_sweeps, 0.0)
    flat0 = obj.env_export()
    obj.env_import(flat0)
    torch.cuda.synchronize()
    say(f"start environment: {n} {prec} sweeps from the identity boundary, corner-spectrum change over the last "
        f"one {delta:.2e}")

    for i in range(args.warmup):
        obj.energy_grad(h, args.grad_sweeps, args.ckpt)
        say(f"warmup step {i} done")
    obj.kernel_timing_enable(True, stride=args.timing_stride)
    e, dA, dt = time_steps(obj, h, args, args.steps)
    timing = obj.kernel_timing()
    obj.kernel_timing_enable(False)
    evals_per_s = args.steps / dt
    sweeps_per_s = time_sweeps(obj, flat0, args.fwd_sweeps)
    say(f"forward sweeps: {sweeps_per_s:.3f} sweeps/s")
    obj.close()
    del obj
    torch.cuda.empty_cache()

    # the other precisions on the same start environment; FP64 is the
    # reference of the error columns (it matches the oracle to 1e-10)
    legs = {prec: {"evals_per_s": evals_per_s, "ms_per_step": 1e3 * dt / args.steps, "sweeps_per_s": sweeps_per_s,
                   "energy": e, "_g": dA}}
    for p in [x for x in args.legs.split(",") if x and x != prec]:
        o = context(p)
        o.env_import(flat0)
        o.energy_grad(h, args.grad_sweeps, args.ckpt)
        say(f"{p} warmup step done")
        ep, gp, dtp = time_steps(o, h, args, args.leg_steps)
        legs[p] = {"evals_per_s": args.leg_steps / dtp, "ms_per_step": 1e3 * dtp / args.leg_steps,
                   "sweeps_per_s": time_sweeps(o, flat0, max(1, args.fwd_sweeps // 2)), "energy": ep, "_g": gp}
        o.close()
        del o
        torch.cuda.empty_cache()
    ref = legs.get("fp64")
    for p, v in legs.items():
        if ref is not None:
            v["energy_rel_err_vs_fp64"] = abs(v["energy"] - ref["energy"]) / abs(ref["energy"])
            v["grad_rel_err_vs_fp64"] = float((v["_g"] - ref["_g"]).norm() / ref["_g"].norm())
            v["speedup_vs_fp64"] = v["evals_per_s"] / ref["evals_per_s"]
    gnorm = float(dA.norm())
    for v in legs.values():
        v.pop("_g")

    dom = max(timing, key=lambda k: timing[k][0])
    ms, launches, flops, nbytes = timing[dom]
    total_ms = sum(v[0] for v in timing.values())
    roof = roofline_of(dom, ms, launches, flops, nbytes)
    roof.update({"traffic": measured_traffic(dom), "kernel": dom, "launches": int(launches),
                 "algorithmic_bytes_per_launch": nbytes / launches if launches else None,
                 "event_sample_stride": args.timing_stride,
                 "avg_launch_us": 1e3 * ms / launches if launches else None,
                 "share_of_timed_kernels": ms / total_ms if total_ms else None,
                 "classes": {k: dict(ms=v[0], launches=int(v[1]), **{kk: vv for kk, vv in
                                     roofline_of(k, *v).items() if kk in ("bound", "achieved", "unit", "frac")})
                             for k, v in timing.items() if v[1] > 0}})

    cpu = None
    if not args.no_cpu_baseline:
        say("CPU oracle sample")
        cpu = cpu_baseline(args.cpu_threads, args.grad_sweeps)

    out = {
        "metric": METRIC,
        "value": evals_per_s,
        "unit": "energy-grad evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": prec,
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "cell": "2x2", "p": 2, "D": 8, "chi_E": chi, "chi_I": chi,
                   "sweeps_per_eval": args.grad_sweeps, "ckpt_every": args.ckpt,
                   "pre_sweeps": args.pre_sweeps, "start_env_delta": delta,
                   "projectors": projectors_label(args)},
        "sweeps_per_s": sweeps_per_s,
        "energy": e,
        "grad_norm": gnorm,
        "mfma_frac": contraction_mfma(timing, prec),
        "precision_legs": legs,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
