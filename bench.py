#!/usr/bin/env python3
"""Projected secants/s and ms per SAP iteration, fused vs plain.

Headline workload: the trigonometric moment curve with harmonics 1..32
(n = 64), N = 4,000 points (7,998,000 unit secants), FP32 input, projection
to k = 6 from the seeded random orthonormal start, alpha = 0.01 -- the curve
of the paper's Sec. 5 at the scale where both forms of the pass fit one GPU.

A timed step is one SAP iteration: evaluate every secant, reduce to the
FP64-rescored min/argmin, apply the update.  `value` is the fused form's
secants/s (kept pairs x timed iterations / time of the timed region, inputs
resident in HBM); the plain form is reported beside it.  `roofline` is the
fused pair pass's: 4 B of 1/d^2 per pair over its average launch duration,
from the kernel's own dispatch timestamps on the library's stream.

Further legs (extra keys, each with secants/s, ms per iteration and the
roofline fraction of its dominant kernel):
  trig10    the paper's Sec. 5 curve, N = 200, n = 10, FP64, k = 3, plain, 200 iterations
  blob      rotated-image stand-in, N = 8,000, n = 1024, k = 2 / 4 / 8, fused, 300 iterations,
            BF16 Y GEMM (the configuration's) and FP64 Y GEMM
  hyper     the hyperspectral stand-in (N = 20,000, n = 200, k = 10): 100 fused iterations, and
            soft-min fwd + bwd + Adam + QR steps
  torus     N = 40,000, n = 256, k = 16: fused iterations (BF16 and FP64 Y GEMM) and a
            soft-min fwd + bwd
  pca       Algorithm 1's secant-PCA start (trig64 and hyper)
  batch     many small problems per launch: the dimension sweep of Sec. 6.1,
            subsamples of Sec. 6.3, the length threshold of Sec. 7
Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0                  # MI355X HBM3E
VALU_LANE_OPS = 256 * 4 * 16 * 2.4e9   # CUs x SIMDs x lanes x clock: lane-instructions/s (FP32 or FP64)
MFMA_F64_TFLOPS = 78.6                 # MI355X dense FP64 matrix peak


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "pass_trig64_N4000_n64_k6_traffic.txt")
KERNEL_SOURCES = ("paper_1807_03425_amd/csrc/sap_iter.hip", "paper_1807_03425_amd/csrc/sap_common.h",
                  "paper_1807_03425_amd/csrc/sap_api.hip", "paper_1807_03425_amd/csrc/sap_kinst.hip",
                  "paper_1807_03425_amd/csrc/sap_launch.h")


def measured_traffic():
    """HBM bytes per launch of the fused and the plain pair pass, from the
    committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary (each counter scaled
    by what it reads for a device copy of known size), while the kernel
    sources still hash to what was profiled; otherwise None for both."""
    none = {"fused": None, "plain": None}
    try:
        with open(TRAFFIC_PROFILE) as f:
            lines = [l for l in f.read().splitlines() if l and not l.startswith("#") and ":" in l]
    except OSError:
        return none
    kv = {k.strip(): v.strip() for k, v in (l.split(":", 1) for l in lines)}
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    if kv.get("source_sha256") != h.hexdigest():
        return none
    return {form: float(kv[f"{form}_traffic_bytes_per_launch"].split()[0]) if f"{form}_traffic_bytes_per_launch" in kv
            else None for form in ("fused", "plain")}


def time_run(torch, ctx, steps, warmup, prof_steps):
    """sap_run timed from the seeded start: wall clock and events around
    the run, then the per-kernel durations of a second, profiled run."""
    dev = torch.device("cuda:0")
    m = steps + 1
    out = dict(min=torch.empty(m, dtype=torch.float64, device=dev),
               ij=torch.empty((m, 2), dtype=torch.int64, device=dev),
               certified=torch.empty(m, dtype=torch.int32, device=dev))
    P0 = ctx.get_P()
    if warmup:
        ctx.run(warmup)
    ctx.set_P(P0)                                   # the timed run starts at the seeded P0
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    ctx.run(steps, out=out)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = e0.elapsed_time(e1)
    P_final = ctx.get_P().cpu().numpy()
    ctx.set_P(P0)
    ctx.profile(True)
    ctx.run(prof_steps)
    prof = ctx.profile_read()
    ctx.profile(False)
    return dict(wall_s=wall, event_ms=ev_ms, trace={k: v.cpu().numpy() for k, v in out.items()},
                P_final=P_final, profile=prof)


def sap_leg(torch, np, w, form, steps, warmup, gemm="f64", prof_steps=None, keep=False):
    """One workload through sap_run: throughput, per-kernel durations and the
    pair pass's roofline (HBM: 4 B of 1/d^2 per pair fused, n x dtype bytes
    per stored secant plain)."""
    from paper_1807_03425_amd import SapContext
    dev = torch.device("cuda:0")
    X = torch.from_numpy(w.X).to(dev)
    t = time.perf_counter()
    ctx = SapContext(X, torch.from_numpy(w.P0), form=form, alpha=w.alpha, gemm=gemm)
    torch.cuda.synchronize()
    init_s = time.perf_counter() - t
    info = ctx.info()
    r = time_run(torch, ctx, steps, warmup, prof_steps or min(steps, 200))
    pairs = info["n_pairs"]
    tsec = max(r["wall_s"], r["event_ms"] / 1e3)
    prof = r["profile"]
    kern = {k: v["ms"] * 1e3 / v["launches"] for k, v in prof.items() if v["launches"]}
    es = w.X.dtype.itemsize
    pass_us = kern.get("pass")
    bytes_launch = 4 * pairs if form == "fused" else es * w.n * pairs
    out = dict(
        workload=f"{w.name}: N={w.N}, n={w.n}, k={w.k}, {w.X.dtype}, {form}, gemm={gemm}",
        pairs=pairs, iters=steps, secants_per_s=pairs * steps / tsec, ms_per_iter=tsec * 1e3 / steps,
        init_s=init_s, certified_frac=float(np.mean(r["trace"]["certified"] == 1)),
        kernel_us_per_launch=kern, n_close=info["n_close"], e_abs=info["e_abs"],
        final_min=float(r["trace"]["min"][-1]))
    if pass_us:
        gbs = bytes_launch / (pass_us * 1e-6) / 1e9
        out["roofline"] = dict(bound="hbm", achieved=gbs, peak=HBM_PEAK_GBS, unit="GB/s",
                               frac=gbs / HBM_PEAK_GBS, kernel=f"sap::k_pass<{w.k}, "
                               f"{'float' if es == 4 else 'double'}, {'true' if form == 'fused' else 'false'}>",
                               bytes_per_launch=bytes_launch, avg_launch_us=pass_us)
        if form == "fused":
            # key arithmetic per pair: K subtractions, K FMAs, a multiply, a min
            valu = (2 * w.k + 2) * pairs
            out["roofline_valu"] = dict(bound="alu", lane_instr_per_launch=valu,
                                        achieved=valu / (pass_us * 1e-6) / 1e12,
                                        peak=VALU_LANE_OPS / 1e12, unit="T lane-instr/s",
                                        frac=valu / (pass_us * 1e-6) / VALU_LANE_OPS)
    if keep:
        out["_ctx"], out["_run"] = ctx, r
    else:
        ctx.close()
    return out


def softmin_slots(K):
    """Vector issue slots per pair of the soft-min passes, counting the
    method's own work (a transcendental -- sqrt, rsq, exp2 -- as 4):
      forward:  K subtractions + K FMAs (||y_i - y_j||^2), a multiply by
                1/d^2, a select of masked pairs, sqrt, min, and for the sum
                an FMA, exp2 and an add: 2K + 14;
      backward: the same 2K for the norm, then multiply, rsq, multiply,
                FMA, exp2, two multiplies, two compares and a select for the
                weight, and the column side's K FMAs (z_j += a (y_j - y_i)):
                3K + 16.  The row side's contraction sum_j a_ij y_j (2K flops
                per pair) runs on the FP64 matrix cores and is priced there
                (softmin_bwd_flops)."""
    return 2 * K + 14, 3 * K + 16


def softmin_bwd_flops(K):
    """FP64 matrix-core flops per pair of the backward's row-side contraction."""
    return 2 * K


def softmin_leg(torch, np, w, tau, steps, warmup, adam=True):
    """ms per soft-min optimisation step (fwd + bwd (+ Adam + QR)) and the
    library's per-kernel split."""
    from paper_1807_03425_amd import SapContext, SoftMinSecant
    dev = torch.device("cuda:0")
    t = time.perf_counter()
    ctx = SapContext(torch.from_numpy(w.X).to(dev), torch.from_numpy(w.P0), form="fused")
    torch.cuda.synchronize()
    init_s = time.perf_counter() - t
    info = ctx.info()
    P = torch.nn.Parameter(torch.from_numpy(w.P0.astype(np.float32)).to(dev))
    opt = torch.optim.Adam([P], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)

    def one():
        opt.zero_grad(set_to_none=False)
        L = SoftMinSecant.apply(P, ctx, tau)
        L.backward()
        if adam:
            opt.step()
            with torch.no_grad():
                Q, R = torch.linalg.qr(P.detach().double())
                sg = torch.where(torch.diagonal(R) < 0, -1.0, 1.0).to(Q.dtype)
                P.copy_((Q * sg.unsqueeze(0)).float())
        return L

    losses = []
    for _ in range(warmup):
        losses.append(one().detach())
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        losses.append(one().detach())
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = max(e0.elapsed_time(e1), wall * 1e3) / steps
    ctx.profile(True)
    nprof = min(steps, 10)
    for _ in range(nprof):
        one()
    prof = ctx.profile_read()
    ctx.profile(False)
    ctx.close()
    pairs = info["n_pairs"]
    kern = {k: v["ms"] / max(v["launches"], 1) for k, v in prof.items() if v["launches"]}
    sf, sb = softmin_slots(w.k)
    out = dict(workload=f"{w.name}: N={w.N}, n={w.n}, k={w.k}, tau={tau}"
                        + (", Adam lr=1e-3 + sign-fixed QR retraction" if adam else ", fwd + bwd"),
               pairs=pairs, steps=steps, warmup=warmup, ms_per_step=ms, init_s=init_s,
               loss_first=float(losses[0]), loss_last=float(losses[-1]),
               kernel_ms_per_launch=kern)
    for slot, slots in (("sm_fwd", sf), ("sm_bwd", sb)):
        if slot in kern:
            ach = slots * pairs / (kern[slot] / 1e3)
            out[f"roofline_{slot}"] = dict(bound="alu", achieved=ach / 1e12, peak=VALU_LANE_OPS / 1e12,
                                           unit="T lane-instr/s", frac=ach / VALU_LANE_OPS,
                                           slots_per_pair=slots, traffic=None)
    if "sm_bwd" in kern:
        fl = softmin_bwd_flops(w.k) * pairs / (kern["sm_bwd"] / 1e3)
        out["mfma_sm_bwd"] = dict(bound="mfma", achieved=fl / 1e12, peak=MFMA_F64_TFLOPS, unit="TFLOP/s",
                                  frac=fl / 1e12 / MFMA_F64_TFLOPS, flops_per_pair=softmin_bwd_flops(w.k))
    return out


def pca_leg(torch, np, w):
    from paper_1807_03425_amd import SapContext
    dev = torch.device("cuda:0")
    ctx = SapContext(torch.from_numpy(w.X).to(dev), torch.from_numpy(w.P0), form="fused")
    ctx.pca_init()                      # warm
    t = time.perf_counter()
    _, info = ctx.pca_init(set_P=True)
    wall = time.perf_counter() - t
    r0 = ctx.min_secant()
    ctx.close()
    return dict(workload=f"{w.name}: N={w.N}, n={w.n}, k={w.k}", device_ms=info["ms"], wall_ms=wall * 1e3,
                iters=info["iters"], residual=info["residual"], converged=info["converged"],
                sigma=info["sigma"], min_at_pca_start=r0["min_norm"])


def batch_leg(torch, np, name, X, sets, problems, P0s, iters, set_min_len=None):
    """One batch of small problems in one launch: total secants/s of the run
    kernel, ms per iteration, and the run kernel's VALU fraction (each problem
    is one workgroup: one compute unit of the 256 at most)."""
    from paper_1807_03425_amd import batch_run
    dev = torch.device("cuda:0")
    Xt = torch.from_numpy(X).to(dev)
    batch_run(Xt, sets, problems, P0s, 2, set_min_len=set_min_len)     # warm
    out = batch_run(Xt, sets, problems, P0s, iters, set_min_len=set_min_len)
    st = out["stats"]
    run_s = st["run_ms"] / 1e3
    pairs = st["n_pairs"]
    # per pair and problem: KP subtractions + KP FMAs (FP64), the FP64
    # multiply by 1/d^2, the conversion to the FP32 key, a min
    kp = [2 if k <= 2 else 4 if k <= 4 else 8 if k <= 8 else 12 if k <= 12 else 16
          for k in (q["k"] for q in problems)]
    ppp = [len(sets[q["set"]]) * (len(sets[q["set"]]) - 1) // 2 for q in problems]
    valu = sum(p * (2 * k + 3) for p, k in zip(ppp, kp)) * (iters + 1)
    cert = out["certified"].cpu().numpy()
    mins = out["min"].cpu().numpy()
    return dict(workload=name, problems=len(problems), sets=len(sets), iters=iters,
                pairs_per_eval=pairs, init_ms=st["init_ms"], run_ms=st["run_ms"],
                secants_per_s=pairs * (iters + 1) / run_s, ms_per_iter=st["run_ms"] / (iters + 1),
                certified_frac=float(np.mean(cert == 1)),
                roofline=dict(bound="alu", achieved=valu / run_s / 1e12, peak=VALU_LANE_OPS / 1e12,
                              unit="T lane-instr/s", frac=valu / run_s / VALU_LANE_OPS,
                              note=f"one workgroup per problem: at most {len(problems)} of 256 compute units"),
                final_min_by_problem=[float(v) for v in mins[:, -1]])


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500, help="timed SAP iterations per form (headline)")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--forms", default="fused,plain")
    ap.add_argument("--legs", default="trig10,blob,hyper,torus,pca,batch",
                    help="further legs (comma list; empty = headline only)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="budget of the FP64 CPU oracle baseline (0 disables it)")
    ap.add_argument("--softmin-steps", type=int, default=20,
                    help="timed soft-min optimisation steps on the hyperspectral workload")
    ap.add_argument("--gemms", default="bf16,f64",
                    help="Y GEMMs of the blob and torus legs (comma list of bf16, f32, f64)")
    ap.add_argument("--blob-ks", default="2,4,8", help="projection dimensions of the blob leg")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first copy a MIB-MiB device buffer 3 times (a kernel of known traffic, "
                         "to scale rocprofv3 FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU: this build runs the SAP pass on a single "
              f"MI355X and has no multi-GPU path (asked for --gpus {args.gpus}, "
              f"WORLD_SIZE={world}).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import sap_inputs

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    if args.calibrate_copy > 0:
        nb = args.calibrate_copy * (1 << 20)
        src = torch.ones(nb // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: 3 copies of {nb} bytes")
        del src, dst
    w = sap_inputs.make("trig64")
    forms = [f for f in args.forms.split(",") if f]
    res = {}
    for form in forms:
        r = sap_leg(torch, np, w, form, args.steps, args.warmup, keep=True)
        log(f"{form}: {args.steps} iterations, {r['ms_per_iter'] * 1e3:.1f} us/iter, "
            f"pass {r['kernel_us_per_launch'].get('pass', 0):.2f} us")
        res[form] = r
    head = "fused" if "fused" in res else forms[0]
    hs = res[head]
    traffic = measured_traffic()
    roofline = dict(hs["roofline"], traffic=traffic.get(head),
                    valu_frac=hs.get("roofline_valu", {}).get("frac"))

    accuracy = {}
    if "fused" in res and "plain" in res:
        a, b = res["fused"]["_run"]["trace"], res["plain"]["_run"]["trace"]
        same = a["ij"] == b["ij"]
        first_diff = int(np.argmin(same.all(axis=1))) if not same.all() else None
        upto = first_diff if first_diff is not None else len(a["min"])
        accuracy["fused_vs_plain"] = dict(
            identical_argmin_trace=first_diff is None, first_divergence=first_diff,
            max_abs_dmin_before_divergence=float(np.max(np.abs(a["min"][:upto] - b["min"][:upto])))
            if upto else None)

    cpu = None
    if args.cpu_seconds > 0:
        import oracle        # CPU baseline leg: the FP64 oracle, untuned
        cores = oracle.num_threads()
        log(f"cpu baseline: FP64 oracle on {cores} threads, budget {args.cpu_seconds}s")
        P = w.P0.copy()
        it = 0
        t0 = time.perf_counter()
        while True:
            m = oracle.min_secant(w.X, P)
            s, _ = oracle.unit_secant(w.X, m["i"], m["j"])
            P, _ = oracle.step(P, s, w.alpha)
            it += 1
            if time.perf_counter() - t0 >= args.cpu_seconds:
                break
        dt = time.perf_counter() - t0
        cpu = dict(value=m["n_pairs"] * it / dt, unit="secants/s", cores=cores, kind="oracle",
                   sample=f"{it} full SAP iterations (all {m['n_pairs']} secants each, "
                          f"FP64, explicit unit secants) of the same workload from the seeded start",
                   ms_per_iter=dt * 1e3 / it)
        log(f"cpu baseline: {it} iterations in {dt:.1f}s")
        # accuracy of the timed GPU runs: the oracle scores each form's final P
        for form, r in res.items():
            tr = r["_run"]["trace"]
            ref = oracle.min_secant(w.X, r["_run"]["P_final"])
            gmin, gij = tr["min"][-1], tuple(tr["ij"][-1])
            accuracy[form] = dict(
                final_min_gpu=float(gmin), final_min_oracle=ref["r_min"],
                rel_err=abs(gmin - ref["r_min"]) / ref["r_min"],
                argmin_match=gij == (ref["i"], ref["j"]),
                oracle_gap_to_runner_up=ref["r_second"] - ref["r_min"])
    for r in res.values():
        r["_ctx"].close()
        del r["_ctx"], r["_run"]
    torch.cuda.synchronize()

    line = dict(
        metric="projected secants/sec + ms per SAP iteration, fused vs plain at stated accuracy",
        value=hs["secants_per_s"], unit="secants/s", n_gpus=1, steps=args.steps,
        warmup=args.warmup, ms_per_step=hs["ms_per_iter"], higher_is_better=True,
        scaling="weak", vs_baseline=None, dtype="f32",
        data="synthetic",
        config=dict(workload="trig moment curve, harmonics 1..32 (n=64), N=4000, FP32, k=6, "
                             "alpha=0.01, seeded random orthonormal start",
                    form=head, pairs=hs["pairs"],
                    arithmetic="FP32 coarse pass; FP64 GEMM (fused), FP64 rescoring and update"),
        roofline=roofline, cpu_baseline=cpu, forms=res, accuracy=accuracy,
    )
    if "plain" in res:
        line["roofline_plain"] = dict(res["plain"]["roofline"], traffic=traffic.get("plain"))
        if "fused" in res:
            line["fused_over_plain"] = res["fused"]["secants_per_s"] / res["plain"]["secants_per_s"]

    legs = [l for l in args.legs.split(",") if l]
    gemms = [g for g in args.gemms.split(",") if g]
    if "trig10" in legs:
        log("leg trig10 (paper Sec. 5 curve, plain FP64, 200 iterations)")
        line["trig10"] = sap_leg(torch, np, sap_inputs.make("trig10"), "plain", 200, 5)
    if "blob" in legs:
        line["blob"] = {}
        for k in [int(v) for v in args.blob_ks.split(",") if v]:
            for g in gemms:
                log(f"leg blob k={k} (fused, {g} Y GEMM, 300 iterations)")
                line["blob"][f"k{k}_{g}"] = sap_leg(torch, np, sap_inputs.make("blob", k=k), "fused", 300, 5,
                                                    gemm=g)
    if "hyper" in legs:
        wh = sap_inputs.make("hyper")
        log("leg hyper: fused iterations")
        line["hyper_iterations"] = sap_leg(torch, np, wh, "fused", 100, 3)
        if args.softmin_steps > 0:
            log("leg hyper: soft-min optimisation steps")
            line["softmin"] = softmin_leg(torch, np, wh, 0.01, args.softmin_steps, 3)
            log(f"soft-min: {line['softmin']['ms_per_step']:.3f} ms/step")
    if "torus" in legs:
        wt = sap_inputs.make("torus")
        line["torus"] = {}
        for g in gemms:
            log(f"leg torus: fused iterations, {g} Y GEMM")
            line["torus"][f"iterations_{g}"] = sap_leg(torch, np, wt, "fused", 100, 3, gemm=g, prof_steps=20)
        log("leg torus: soft-min fwd + bwd")
        line["torus"]["softmin"] = softmin_leg(torch, np, wt, 0.01, 3, 1, adam=False)
    if "pca" in legs:
        line["pca_init"] = {}
        for nm in ("trig64", "hyper"):
            log(f"leg pca: {nm}")
            line["pca_init"][nm] = pca_leg(torch, np, sap_inputs.make(nm))
    if "batch" in legs:
        line["batch"] = {}
        ks = list(range(1, 11))
        log("leg batch: dimension sweep (Sec. 6.1)")
        X = np.concatenate([sap_inputs.embedded_manifold(kd, 256, 10 + e)
                            for e, kd in enumerate(("curve", "torus", "sphere"))])
        sets = [np.arange(e * 256, (e + 1) * 256, dtype=np.int32) for e in range(3)]
        probs = [dict(set=s, k=k) for s in range(3) for k in ks]
        line["batch"]["sweep"] = batch_leg(
            torch, np, "curve / 2-torus / 3-sphere in R^15, 256 points each, k = 1..10, 100 iterations",
            X, sets, probs, sap_inputs.sweep_starts(15, [q["k"] for q in probs], 21), 100)
        log("leg batch: subsample ensemble (Sec. 6.3)")
        wh = sap_inputs.make("hyper")
        sets = sap_inputs.subsample_sets(wh.N, 10, 512, seed=63)
        probs = [dict(set=s, k=k) for s in range(10) for k in ks]
        line["batch"]["subsamples"] = batch_leg(
            torch, np, "hyperspectral stand-in (N=20000, n=200, FP32): 10 x 512-point subsamples, "
                       "k = 1..10, 100 iterations",
            wh.X, sets, probs, sap_inputs.sweep_starts(wh.n, [q["k"] for q in probs], 64), 100)
        log("leg batch: length threshold (Sec. 7)")
        Xn, _ = sap_inputs.trig_curve(512, 5, seed=71, noise=0.1)
        Xc, _ = sap_inputs.trig_curve(512, 5, seed=71)
        X = np.concatenate([Xc, Xn])
        sets = [np.arange(512, dtype=np.int32), np.arange(512, 1024, dtype=np.int32),
                np.arange(512, 1024, dtype=np.int32)]
        # k = 1..9: at k = n = 10 the projection is the identity and every
        # pair ties at r = 1
        probs = [dict(set=s, k=k) for s in range(3) for k in range(1, 10)]
        line["batch"]["threshold"] = batch_leg(
            torch, np, "trig curve R^10, 512 points: clean, noisy (sigma 0.1), noisy with l = 2; "
                       "k = 1..9, 100 iterations",
            X, sets, probs, sap_inputs.sweep_starts(10, [q["k"] for q in probs], 72), 100,
            set_min_len=[0.0, 0.0, 2.0])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
