"""Throughput benchmark: Monte Carlo evaluation of the 10x2 lattice Burgers
functional integral (integrand evaluations per second) on one MI355X.

One step = one pass of the whole path over the workload: the resident plan
(subvolume descriptors and work items already in HBM) is replayed as a captured
graph (queue reset, persistent Monte Carlo kernel, ordered per-subvolume merge),
the per-subvolume records are copied to the host and finalized into Z, C(r) and
their error bars.  Both arithmetic forms run on the same points: FP64, and FP32
action/exp with a shifted weight and FP64 sums.  The JSON line reports the form
named in config.form as `value`, the other form beside it, the FP32-vs-FP64
deviation, the hot kernel against the VALU issue roofline, and the FP64 CPU
oracle timed on a bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload burgers10x2]
"""
from __future__ import annotations

import argparse
import gc
import itertools
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402

METRIC = "integrand evals/s @10x2 lattice, FP32-eval vs FP64 at rel err 1e-3; p99 latency"

# VALU issue roofline.  MI355X: 256 CUs at 2.4 GHz; the published vector peaks
# (FP64 78.6 TFLOP/s, FP32 157.3 TFLOP/s) fix the issue width per clock and CU:
# 64 lanes for FP64 arithmetic, and 128 lanes for FP32 arithmetic.  The
# independent-chain probe (microbench/issue_rates.hip) puts 32-bit integer
# multiplies (v_mad_u64_u32, v_mul_lo/hi_u32) and conversions at the FP64 rate,
# 32-bit logic (v_xor_b32, v_bitop3_b32) and non-packed v_fma_f32 at 1.6-1.7x
# it, and FP32 transcendentals at half of it.  Work is counted in FP64-rate lane
# slots: 1 per 64-lane-class instruction, 1/2 per 128-lane-class instruction,
# 2 per transcendental.
SLOT = {"f64": 1.0, "mul32": 1.0, "cvt": 1.0, "f32": 0.5, "logic32": 0.5, "trans": 2.0}
EXP64_OPS = 19              # FP64 exp routine: scale, round, 2 reductions, 11 poly, ldexp, checks
PEAK_SLOTS = 256 * 64 * 2.4e9   # FP64-rate lane slots per second (= FP64 FMA/s)
PEAK_FP64 = 78.6e12


def valu_slots_per_eval(nx: int, nt: int, prec: str, observable: str = "anchor",
                        pairs: bool = False) -> float:
    """FP64-rate lane slots one evaluation needs (algorithmic instruction counts):
      Philox4x32-10: per block 10 rounds x (2 wide 32x32 multiplies + 2 xor3)
      point map:     per variable one u32->float conversion and one fma
      action:        per site 6 (two sums/differences, three fma, one fma into S), + 1
      weight:        FP64 exp routine; FP32 form: multiply, exp2, widen to FP64
      sums:          w, w^2 (2) + p_r scale x w (1) + per r: product, add, 2 fma (4)
                     FP32 form: the product in FP32, then one widening per r
      averaged observable: r = 0 .. nx/2 only; p_r = sum over the sites and time
                     slices of u_m u_{m+r} (one fma per term, the pair at r = nx/2
                     counted once and doubled)
      antithetic pairs: one Philox evaluation per pair of points; per pair the
                     two weights averaged, t = p_0 w for each point, per r the
                     mean of the two products (product, fma, halving) and its
                     three sums: FP64 3 + 3 nr per evaluation (FP32 form: the
                     combination in FP32, one widening per r, 2.5 + 2.75 nr)"""
    d, nb = nx * nt, (nx * nt + 3) // 4
    avg = observable == "averaged"
    nr = nx // 2 + 1 if avg else nx
    f = SLOT["f64"] if prec == "fp64" else SLOT["f32"]
    philox = nb * 10 * (2 * SLOT["mul32"] + 2 * SLOT["logic32"])
    if pairs:
        philox /= 2
    if prec == "fp64":
        mapping = d * (SLOT["cvt"] + SLOT["f64"])
        action = (6 * d + 1) * SLOT["f64"]
        weight = EXP64_OPS * SLOT["f64"]
        sums = ((3 + 3 * nr) if pairs else (3 + 4 * nr)) * SLOT["f64"]
    else:
        mapping = d * (SLOT["cvt"] * 0.5 + SLOT["f32"])   # u32->f32 is a 32-bit op
        action = (6 * d + 1) * SLOT["f32"]
        weight = SLOT["f32"] + SLOT["trans"] + SLOT["cvt"] + SLOT["f32"]  # (sigma-S)*log2e, exp2, widen, compare
        if pairs:
            sums = (1 + 1.5 * nr) * SLOT["f64"] + nr * (0.75 * SLOT["f32"] + 0.5 * SLOT["cvt"]) \
                + 1.5 * SLOT["f32"]
        else:
            sums = (2 + 3 * nr) * SLOT["f64"] + nr * (SLOT["f32"] + SLOT["cvt"]) + SLOT["f32"]
    observable_terms = 0.0
    if avg:
        half = nx % 2 == 0 and nx > 1
        terms = sum(nx // 2 if half and 2 * r == nx else nx for r in range(nr))
        observable_terms = (nt * terms + (1 if half else 0)) * f
    return philox + mapping + action + weight + sums + observable_terms


def fp64_flops_per_eval(nx: int, nt: int, pairs: bool = False) -> float:
    """FP64 floating-point operations (FMA = 2) of one FP64-form evaluation:
    map 2d, action 10 per site + 1, exp ~30, sums 2 + 1 + 7 per r (+ w^2 fma);
    antithetic pairs: per pair the weights averaged (2), t of each point (2),
    per r the halved mean of the products (4) and its sums (5), and w, w^2 (3),
    i.e. 3.5 + 4.5 nx per evaluation."""
    d = nx * nt
    sums = (3.5 + 4.5 * nx) if pairs else (1 + 2) + 1 + 7 * nx
    return 2 * d + 10 * d + 1 + 30 + sums


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="burgers10x2", choices=sorted(workloads.WORKLOADS))
    ap.add_argument("--headline", default="fp64", choices=["fp64", "fp32"],
                    help="form reported as value (fp64: the paper's double-precision "
                         "arithmetic; fp32: FP32 action/exp, FP64 sums)")
    ap.add_argument("--cpu-samples-log2", type=int, default=None,
                    help="oracle sample: first 2^k samples of every subvolume (default: about "
                         "2^29 x 20/d evaluations in all, 10-15 s on 16 host threads)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="length of the Poisson serving run (0 skips it)")
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-max-samples-per-thread", type=int, default=0,
                    help="cap on samples per thread of served items (0: the server's 128)")
    ap.add_argument("--adaptive-budget-log2", type=int, default=36,
                    help="evaluation budget of each adaptive 10x2 run (0 skips them)")
    ap.add_argument("--adaptive-target-budget-log2", type=int, default=40,
                    help="budget of the holdout-confirmed time-to-target adaptive runs with the "
                         "averaged observable (0 skips them)")
    ap.add_argument("--adaptive-scale-budget-log2", type=int, default=39,
                    help="budget of the large adaptive run (over a million leaves; 0 skips it)")
    ap.add_argument("--no-observable-leg", action="store_true",
                    help="skip the translation-averaged observable leg")
    ap.add_argument("--no-sampler-leg", action="store_true",
                    help="skip the Gaussian-proposal sampler leg")
    ap.add_argument("--no-antithetic-leg", action="store_true",
                    help="skip the antithetic-pair leg")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="also run one device copy of this size (counter calibration)")
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_1803_07560_amd",
                                                         "tuned_gfx950.json"))
    return ap.parse_args()


def run_form(bfi, torch, ctx, lat, sv, w, prec, steps, warmup, stream):
    """Time `steps` steps of one form: each step replays the plan's graph (queue
    reset, Monte Carlo kernel, merge, copy of the records to a device buffer),
    copies the records to the host and finalizes them.  The timed steps are
    pipelined: step i+1 is enqueued before step i's records come back (on a
    second stream, into pinned host memory) and are finalized, so the GPU does
    not wait for the host between steps.  Two device buffers alternate (the plan
    keeps one captured replay per buffer); a buffer is reused only after its
    copy has been waited for.  Replay durations come from events recorded on the
    launch stream around every replay."""
    plan = bfi.bfi_plan_create(ctx, lat, prec, sv, bfi.launch(use_graph=1))
    try:
        info = bfi.bfi_plan_info(plan)
        shape = (len(sv), 4 + 3 * w.nx)
        dev = [torch.empty(shape, dtype=torch.float64, device="cuda") for _ in range(2)]
        host = [torch.empty(shape, dtype=torch.float64, pin_memory=True) for _ in range(2)]
        copy_stream = torch.cuda.Stream()
        copied = [torch.cuda.Event() for _ in range(2)]
        # first use of each stream before any launch: a stream's hardware queue
        # is set up when it first takes work, which would interrupt a running
        # kernel (its waves saved and restored) and count against that launch
        for st in (stream, copy_stream):
            with torch.cuda.stream(st):
                host[0].copy_(dev[0], non_blocking=True)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(steps)]

        def launch(i, timed):
            b = i % 2
            if timed:
                ev[i][0].record(stream)
            bfi.bfi_plan_run(plan, w.seed, dev[b], stream)
            done = torch.cuda.Event()
            done.record(stream)
            if timed:
                ev[i][1].record(stream)
            copy_stream.wait_event(done)
            with torch.cuda.stream(copy_stream):
                host[b].copy_(dev[b], non_blocking=True)
                copied[b].record(copy_stream)

        def finish(i):
            b = i % 2
            copied[b].synchronize()
            return bfi.bfi_finalize(lat, sv, host[b].numpy())

        # collector paused from here to the end of the timed steps (a collection
        # before the timed loop would idle the GPU and let its clock drop)
        gc.collect()
        gc.disable()
        # warm-up in the timed loop's pattern (a copy overlapping the next
        # launch, which the first time stalled that launch by ~6 ms)
        if warmup > 0:
            launch(0, False)
            for i in range(1, warmup):
                launch(i, False)
                finish(i - 1)
            finish(warmup - 1)
        torch.cuda.synchronize()
        step_end = []
        t0 = time.perf_counter()
        launch(0, True)
        for i in range(1, steps):
            launch(i, True)
            res = finish(i - 1)
            step_end.append(time.perf_counter())
        res = finish(steps - 1)
        step_end.append(time.perf_counter())
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        kernel_ms = [a.elapsed_time(b) for a, b in ev]
        part = host[(steps - 1) % 2].numpy().copy()
    finally:
        gc.enable()
        bfi.bfi_plan_destroy(plan)
    evals = info["n_evals"]
    step_ms = 1e3 * np.diff(np.concatenate([[t0], step_end]))
    return {"evals_per_s": steps * evals / (t1 - t0), "ms_per_step": 1e3 * (t1 - t0) / steps,
            "step_ms_median": float(np.median(step_ms)), "step_ms_max": float(np.max(step_ms)),
            "step_ms_each": [round(float(x), 3) for x in step_ms[:200]],
            "kernel_ms_each": [round(float(x), 3) for x in kernel_ms[:200]],
            "kernel_ms": float(np.mean(kernel_ms)), "kernel_ms_min": float(np.min(kernel_ms)),
            "kernel_ms_median": float(np.median(kernel_ms)),
            "evals_per_step": evals, "result": res, "partials": part,
            "launch": {k: info[k] for k in ("samples_per_thread", "block", "persistent",
                                            "use_graph")}, "n_items": info["n_items"]}


def serve_leg(bfi, ctx, seconds, rate, warmup_s=1.0, max_samples_per_thread=0, alone=50):
    """Poisson arrivals of correlation requests (lattice uniform over 4x2, 8x2,
    10x2, 16x4; nu log-uniform in [0.05, 2]; budgets 2^U(16,26)); FP32 form.
    Latency is submit-to-result as timed by the server; requests arriving in the
    first `warmup_s` seconds are served but not counted.  Afterwards `alone`
    requests sampled from the stream (numpy PCG64(2)) run again one at a time on
    a fresh server: each result must be bit-identical to its result in the mix."""
    reqs = workloads.serving_requests(rate, seconds, seed=1)
    cfg = bfi.server_config(memory_budget=8 << 30, max_requests=256,
                            max_samples_per_thread=max_samples_per_thread)
    srv = bfi.bfi_server_create(ctx, cfg)
    try:
        t0 = time.perf_counter()
        tickets = []
        for r in reqs:
            while True:
                dt = r.arrival_s - (time.perf_counter() - t0)
                if dt <= 0:
                    break
                time.sleep(min(dt, 0.001))
            tickets.append(bfi.bfi_server_submit(srv, bfi.request(
                bfi.lattice(r.nx, r.nt, nu=r.nu, D=r.D), "fp32", r.seed, r.box, r.split_log2,
                r.budget)))
        done = [bfi.bfi_server_wait(srv, t, 120.0) for t in tickets]
        t1 = time.perf_counter()
        st = bfi.bfi_server_stats_get(srv)
    finally:
        bfi.bfi_server_destroy(srv)
    lat = [x[1] for x in done]
    counted = np.array([x for x, r in zip(lat, reqs) if r.arrival_s >= warmup_s])
    evals = sum(r.budget for r in reqs)
    # the same requests alone: bit-identical results
    pick = np.random.Generator(np.random.PCG64(2)).choice(len(reqs), size=min(alone, len(reqs)),
                                                          replace=False)
    same = 0
    srv = bfi.bfi_server_create(ctx, cfg)
    try:
        for i in sorted(pick):
            r = reqs[i]
            t = bfi.bfi_server_submit(srv, bfi.request(
                bfi.lattice(r.nx, r.nt, nu=r.nu, D=r.D), "fp32", r.seed, r.box, r.split_log2,
                r.budget))
            res = bfi.bfi_server_wait(srv, t, 120.0)[0]
            mix = done[i][0]
            same += int(res["log_Z"] == mix["log_Z"] and np.array_equal(res["C"], mix["C"])
                        and np.array_equal(res["C_err"], mix["C_err"]))
    finally:
        bfi.bfi_server_destroy(srv)
    if same != len(pick):
        print(f"bench: WARNING: {len(pick) - same} of {len(pick)} requests differ alone vs mixed",
              file=sys.stderr, flush=True)
    return {"requests": len(reqs), "counted": int(counted.size), "rate_hz": rate,
            "seconds": seconds, "warmup_seconds": warmup_s,
            "p50_ms": float(np.percentile(counted, 50) * 1e3),
            "p99_ms": float(np.percentile(counted, 99) * 1e3),
            "max_ms": float(counted.max() * 1e3), "evals_per_s": evals / (t1 - t0),
            "gpu_busy_frac": st["busy_seconds"] / (t1 - t0), "steps": st["steps"],
            "step_ms_mean": 1e3 * st["busy_seconds"] / max(st["steps"], 1),
            "alone_vs_mixed_bit_identical": f"{same}/{len(pick)}", "form": "fp32"}


def adaptive_leg(bfi, ctx, budget_log2, nus=(0.1, 0.5, 1.0), observables=("anchor", "averaged"),
                 forms=("fp32",), holdout_forms=(), confirm=False, target=1e-3, seeds=(1,)):
    """10x2 lattice, D = 1, box [-4,4]^20: error-driven bisection from the
    1024-subvolume partition at 2^10 samples per leaf, per-leaf counts in
    [2^10, 2^22], target max_r sigma_C(r)/|C(0)| <= 1e-3 with an effective
    sample size of at least 100, in the given forms, budget 2^budget_log2
    evaluations per value of nu, each round at least 1/32 of it; split statistics
    from the first 2^16 samples of each leaf; the anchored product of the paper
    and the translation-averaged one.  With `confirm`, the stop is confirmed on a
    holdout pass (the leaves sampled afresh under a seed of their own, at most
    one check per round): status BFI_OK then means a holdout pass met the target
    and `seconds` is the time to it; BFI_EBUDGET reports the last holdout error.
    Without it, BFI_OK means the running estimate met the target.  For runs in
    `holdout_forms` the final partition is also evaluated on a fresh pass (each
    leaf's stream continued over n more samples, which no refinement decision
    has seen): `holdout_rel_err` is that pass's max_r sigma_C(r)/|C(0)|, free of
    the selection that makes the stopping estimate optimistic."""
    out = []
    for form, observable, nu, seed in itertools.product(forms, observables, nus, seeds):
        cfg = bfi.adaptive_config(target_rel_err=target, max_evals=1 << budget_log2,
                                  n_min=1 << 10, n_max=1 << 22, split_log2=10,
                                  max_rounds=128, refine_fraction=0.5,
                                  round_evals=max(1 << 24, (1 << budget_log2) >> 5),
                                  split_samples=1 << 16, holdout=confirm)
        t0 = time.perf_counter()
        r = bfi.bfi_integrate_adaptive(ctx, bfi.lattice(10, 2, nu=nu, observable=observable),
                                       form, seed, -4.0, 4.0, cfg, leaf_capacity=1 << 22)
        dt = time.perf_counter() - t0
        print(f"bench: adaptive {form} {observable} nu={nu} seed {seed} target {target:g}: {r['status']} "
              f"rel_err {r['rel_err']:.3g} (holdout {r['holdout_rel_err']:.3g}) in {dt:.2f} s",
              file=sys.stderr, flush=True)
        part = r["partition"]
        n = part.n
        rec = {"form": form, "observable": observable, "nu": nu, "seed": seed, "target": target,
               "status": r["status"],
               "stop": "holdout-confirmed" if confirm else "running estimate",
               "rel_err": r["rel_err"], "ess": r["ess"], "rounds": r["rounds"],
               "leaves": r["leaves"], "evals": r["evals"], "seconds": dt,
               "evals_per_s": r["evals"] / dt, "device_seconds": r["device_seconds"],
               "leaf_n_min": int(n.min()), "leaf_n_max": int(n.max()),
               "split_samples": cfg.split_samples}
        if confirm:
            rec["holdout_checks"] = r["holdout_checks"]
            rec["holdout_used"] = r["holdout_used"]
            rec["last_holdout_rel_err"] = r["holdout_rel_err"]
        if form in holdout_forms:
            lat = bfi.lattice(10, 2, nu=nu, observable=observable)
            fresh = bfi.Subvolumes(part.ids, part.lo, part.hi, n, n, lat.d)
            h = bfi.bfi_finalize(lat, fresh, bfi.bfi_eval(ctx, lat, form, seed, fresh))
            rec["holdout_rel_err"] = float(np.max(h["C_err"]) / abs(h["C"][0]))
            rec["holdout_ess"] = float(h["ess"])
            rec["holdout_C_dev"] = float(np.max(np.abs(h["C"] - r["C"])) / abs(r["C"][0]))
            print(f"bench: holdout pass rel_err {rec['holdout_rel_err']:.3g}", file=sys.stderr,
                  flush=True)
        out.append(rec)
    return out


def adaptive_scale_leg(bfi, ctx, budget_log2=39, n_max_log2=18, round_log2=34,
                       split_samples_log2=16):
    """A large adaptive 10x2 run (FP32 form, averaged observable, box [-4,4]^20):
    from 1024 leaves at 2^10 samples, leaves capped at 2^n_max_log2 samples so
    refinement splits, rounds of 2^round_log2 evaluations, the split statistics
    over each leaf's first 2^split_samples_log2 samples, to a budget of
    2^budget_log2 -- over a million leaves.  Reports the whole run's rate and
    the device's share of its wall time (events around each replay of the
    captured round sequence)."""
    cfg = bfi.adaptive_config(target_rel_err=1e-9, max_evals=1 << budget_log2, n_min=1 << 10,
                              n_max=1 << n_max_log2, split_log2=10, max_rounds=1000,
                              refine_fraction=0.5, round_evals=1 << round_log2,
                              split_samples=1 << split_samples_log2)
    t0 = time.perf_counter()
    r = bfi.bfi_integrate_adaptive(ctx, bfi.lattice(10, 2, observable="averaged"), "fp32", 1,
                                   -4.0, 4.0, cfg, leaf_capacity=1)
    dt = time.perf_counter() - t0
    print(f"bench: adaptive scale run: {r['leaves']} leaves, {r['evals']:.3g} evals in {dt:.2f} s "
          f"(device {r['device_seconds']:.2f} s)", file=sys.stderr, flush=True)
    return {"budget": 1 << budget_log2, "n_max": 1 << n_max_log2, "round_evals": 1 << round_log2,
            "split_samples": 1 << split_samples_log2, "rounds": r["rounds"], "leaves": r["leaves"], "evals": r["evals"], "seconds": dt,
            "evals_per_s": r["evals"] / dt, "device_seconds": r["device_seconds"],
            "device_evals_per_s": r["evals"] / r["device_seconds"],
            "wall_over_device": dt / r["device_seconds"],
            "graph_instantiations": r["graph_instantiations"],
            "graph_updates": r["graph_updates"], "form": "fp32", "observable": "averaged"}


def host_path_leg(bfi, ctx, lat, sv, reps=3):
    """The host-array entry `bfi_eval` on the same workload: descriptors and items
    built and uploaded, the kernel run, the records copied back and the device
    buffers freed on every call, so its rate includes PCIe and allocation (median
    of `reps` calls after one warm-up call, per form)."""
    out = {}
    for prec in ("fp64", "fp32"):
        bfi.bfi_eval(ctx, lat, prec, 1, sv)
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            bfi.bfi_eval(ctx, lat, prec, 1, sv)
            ts.append(time.perf_counter() - t0)
        t = float(np.median(ts))
        out[prec] = {"ms": t * 1e3, "evals_per_s": float(np.sum(sv.n)) / t}
    return out


def observable_leg(bfi, torch, ctx, w, sv, steps, warmup, stream, accuracy_log2=26):
    """The translation-averaged product (p_r averaged over every anchor):
    throughput of both forms on the benchmark workload, and on the paper's
    integration range [-1, 1]^20 (2^accuracy_log2 points, 64 subvolumes, FP32
    form) the error bars of both observables on the same points.  The time to
    reach a given error scales as sigma^2 / rate, so the equal-error speedup
    per r is (sigma_anchor / sigma_averaged)^2 * rate_averaged / rate_anchor."""
    lat = bfi.lattice(w.nx, w.nt, nu=w.nu, D=w.D, observable="averaged")
    forms = {}
    for prec in ("fp64", "fp32"):
        print(f"bench: averaged observable {prec}", file=sys.stderr, flush=True)
        f = run_form(bfi, torch, ctx, lat, sv, w, prec, steps, warmup, stream)
        slots = valu_slots_per_eval(w.nx, w.nt, prec, "averaged")
        rate = slots * f["evals_per_step"] / PEAK_SLOTS
        forms[prec] = {"evals_per_s": f["evals_per_s"], "ms_per_step": f["ms_per_step"],
                       "kernel_ms": f["kernel_ms"], "kernel_ms_median": f["kernel_ms_median"],
                       "slots_per_eval": slots, "valu_frac": rate / (f["kernel_ms"] * 1e-3),
                       "valu_frac_median": rate / (f["kernel_ms_median"] * 1e-3)}
    est = {}
    for obs in ("anchor", "averaged"):
        est[obs] = bfi.bfi_integrate(ctx, bfi.lattice(w.nx, w.nt, nu=w.nu, D=w.D, observable=obs),
                                     "fp32", 3, -1.0, 1.0, 6, 1 << accuracy_log2)
    ratio = np.asarray(est["anchor"]["C_err"]) / np.asarray(est["averaged"]["C_err"])
    return {"forms": forms, "paper_range": {
        "box": [-1.0, 1.0], "evals": 1 << accuracy_log2, "form": "fp32",
        "C_anchor": [float(c) for c in est["anchor"]["C"]],
        "C_averaged": [float(c) for c in est["averaged"]["C"]],
        "C_err_ratio": [float(x) for x in ratio]}}


def antithetic_leg(bfi, torch, ctx, w, sv, steps, warmup, stream, accuracy_log2=26):
    """Antithetic pairs: every sample index evaluates the point of its Philox
    words and of the complemented words (its reflection through the subvolume's
    centre), sharing one Philox evaluation.  Throughput of both forms on the
    benchmark workload (the same evaluations: half the sample indices, two
    points each), and the error bars of pairs and single points at equal
    evaluations (2^accuracy_log2, FP32 form) on the paper's range [-1,1]^20 (64
    subvolumes) and on the benchmark box.  Time to a given error scales as
    sigma^2 / rate: the equal-error speedup is
    (sigma_single / sigma_pairs)^2 rate_pairs / rate_single."""
    lat = bfi.lattice(w.nx, w.nt, nu=w.nu, D=w.D, antithetic=True)
    half = bfi.Subvolumes(sv.ids, sv.lo, sv.hi, sv.n // 2, sv.offset, w.d)
    forms = {}
    for prec in ("fp64", "fp32"):
        print(f"bench: antithetic pairs {prec}", file=sys.stderr, flush=True)
        f = run_form(bfi, torch, ctx, lat, half, w, prec, steps, warmup, stream)
        rate = f["evals_per_step"] / (f["kernel_ms"] * 1e-3)
        slots = valu_slots_per_eval(w.nx, w.nt, prec, pairs=True)
        forms[prec] = {"evals_per_s": f["evals_per_s"], "ms_per_step": f["ms_per_step"],
                       "kernel_ms": f["kernel_ms"], "kernel_ms_median": f["kernel_ms_median"],
                       "evals_per_step": f["evals_per_step"], "slots_per_eval": slots,
                       "valu_frac": slots * rate / PEAK_SLOTS}
        if prec == "fp64":
            flops = fp64_flops_per_eval(w.nx, w.nt, pairs=True)
            forms[prec]["fp64_flops_per_eval"] = flops
            forms[prec]["fp64_flop_frac"] = flops * rate / PEAK_FP64
    boxes = []
    for B, k in ((1.0, 6), (w.box, w.split_log2)):
        est = {}
        for kind, anti in (("single", False), ("pairs", True)):
            est[kind] = bfi.bfi_integrate(
                ctx, bfi.lattice(w.nx, w.nt, nu=w.nu, D=w.D, antithetic=anti), "fp32", 5, -B, B,
                k, 1 << accuracy_log2)
        boxes.append({
            "box": [-B, B], "subvolumes": 1 << k, "evals": 1 << accuracy_log2, "form": "fp32",
            "Z_err_ratio": est["single"]["Z_err"] / est["pairs"]["Z_err"],
            "C_err_ratio": [float(a / b) for a, b in zip(est["single"]["C_err"],
                                                         est["pairs"]["C_err"])],
            "Z": [est["single"]["Z"], est["pairs"]["Z"]],
            "Z_err": [est["single"]["Z_err"], est["pairs"]["Z_err"]]})
    return {"forms": forms, "error_at_equal_evals": boxes}


def sampler_leg(bfi, ctx, w, budget_log2=28, alpha=0.9, repeats=3, shells=64, pilot=0.125):
    """The defensive Gaussian-proposal sampler and the sampler in spherical
    coordinates (`shells` equal-width radial shells out to the cube's corners, a
    pilot pass of `pilot` of the budget, then Neyman's allocation) against the
    plain cartesian one on the 10x2 lattice, same budget, FP32 form, on the
    benchmark box [-4,4]^20 and on the paper's range [-1,1]^20: effective
    sample size (sum W)^2 / sum W^2, wall time of the whole call (plan, kernel,
    finalize), and their ratio."""
    lat = bfi.lattice(w.nx, w.nt, nu=w.nu, D=w.D)
    budget = 1 << budget_log2
    out = []
    for B in (w.box, 1.0):
        row = {"box": [-B, B], "evals": budget, "alpha": alpha, "shells": shells,
               "pilot_fraction": pilot}
        for kind in ("plain", "gaussian_mixture", "spherical"):
            best, res = None, None
            for _ in range(repeats):
                t0 = time.perf_counter()
                if kind == "plain":
                    res = bfi.bfi_integrate(ctx, lat, "fp32", 1, -B, B, w.split_log2, budget)
                elif kind == "gaussian_mixture":
                    res = bfi.bfi_integrate_is(ctx, lat, "fp32", 1, -B, B, budget, alpha, 256)
                else:
                    res = bfi.bfi_integrate_sph(ctx, lat, "fp32", 1, B, shells, budget, pilot)
                dt = time.perf_counter() - t0
                best = dt if best is None else min(best, dt)
            row[kind] = {"seconds": best, "evals_per_s": budget / best, "ess": res["ess"],
                         "ess_per_s": res["ess"] / best, "Z": res["Z"], "Z_err": res["Z_err"],
                         "C0": float(res["C"][0]), "C0_err": float(res["C_err"][0])}
        out.append(row)
    return out


def kernel_source_digest():
    """sha256 of the kernel sources: traffic figures apply only to the kernel
    they were measured on."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1803_07560_amd", "csrc")
    for name in ("shape_kernels.hip", "device.hpp", "exp64.hpp", "internal.h"):
        h.update(open(os.path.join(csrc, name), "rb").read())
    return h.hexdigest()


def measured_traffic(workload, form):
    """HBM bytes per launch of mc_kernel from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel calibration), or None
    if the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_source_sha256") != kernel_source_digest():
        return None
    return rec.get("bytes_per_launch", {}).get(form)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, sv, k, k_single=12):
    """The FP64 oracle (plain C, one subvolume per thread at a time) on the first
    2^k samples of every subvolume, on the host's CPU share: the CPUs this
    process may run on, at most 16 (one GPU's share of the box).  Also timed on
    one thread over the first 2^k_single samples.  Returns the baseline and the
    oracle's sums over the sample (with the L1 fields), which the GPU forms are
    then checked against on the same points."""
    import oracle
    sub = sv.subset(np.arange(len(sv)))
    if k is None:
        k = max(int(math.floor(math.log2(2**29 * 20 / w.d / len(sub)))), 1)
    per = min(int(sub.n[0]), 1 << k)
    sub.n[:] = per
    avail = len(os.sched_getaffinity(0))
    threads = max(1, min(16, avail))
    lat = oracle.lattice(w.nx, w.nt, nu=w.nu, D=w.D)
    t0 = time.perf_counter()
    rec = oracle.sums_l1(lat, w.seed, sub.ids, sub.lo, sub.hi, sub.n, sub.offset,
                         nthreads=threads)
    dt = time.perf_counter() - t0
    n = per * len(sub)
    one = sub.subset(np.arange(len(sub)))
    per1 = min(per, 1 << k_single)
    one.n[:] = per1
    t1 = time.perf_counter()
    oracle.sums_l1(lat, w.seed, one.ids, one.lo, one.hi, one.n, one.offset, nthreads=1)
    dt1 = time.perf_counter() - t1
    base = {"value": n / dt, "unit": "evals/s", "cores": threads, "kind": "oracle",
            "sample": f"first 2^{per.bit_length() - 1} samples of each of the {len(sub)} "
                      f"subvolumes ({n} evals, {dt:.1f} s, FP64 scalar C oracle with L1 sums, "
                      f"{threads} pthreads)",
            "cpu_model": cpu_model(), "os_cpu_count": os.cpu_count(), "cpus_available": avail,
            "value_1_thread": per1 * len(one) / dt1,
            "sample_1_thread": f"first 2^{per1.bit_length() - 1} samples of each subvolume "
                               f"({per1 * len(one)} evals, {dt1:.1f} s)"}
    return base, sub, rec


def error_vs_oracle(bfi, ctx, w, sub, rec):
    """Each form on the GPU over the oracle's sample (same points): Z's relative
    error, and the largest C(r) error over its L1 scale sum_s V_s/n_s sum |p_r w| / Z."""
    import oracle
    L = oracle.sums_len(w.nx)
    plain, l1 = rec[:, :L], rec[:, L:]
    ref = oracle.finalize(w.nx, w.d, sub.lo, sub.hi, plain)
    v = np.prod(sub.hi - sub.lo, axis=1) / plain[:, 0]
    scale = np.sum(v[:, None] * l1, axis=0) / np.sum(v * plain[:, 1])
    lat = bfi.lattice(w.nx, w.nt, nu=w.nu, D=w.D)
    out = {"points": int(sub.n.sum()), "oracle_Z": float(ref["Z"]),
           "oracle_C": [float(c) for c in ref["C"]]}
    for prec in ("fp64", "fp64s", "fp32"):
        res = bfi.bfi_finalize(lat, sub, bfi.bfi_eval(ctx, lat, prec, w.seed, sub))
        out[prec] = {"Z_rel": abs(res["log_Z"] - ref["log_Z"]),
                     "C_over_L1_max": float(np.max(np.abs(res["C"] - ref["C"]) / scale))}
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); the "
              "subvolume sharding across GPUs is described in the design notes but not built.",
              file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_1803_07560_amd as bfi

    w = workloads.WORKLOADS[args.workload]
    sv = workloads.uniform_partition(w.d, w.box, w.split_log2, w.budget // w.n_sub)
    lat = bfi.lattice(w.nx, w.nt, nu=w.nu, D=w.D)
    ctx = bfi.bfi_context_create(0)
    if os.path.exists(args.tune_cache):
        bfi.bfi_tune_load(ctx, args.tune_cache)
    stream = torch.cuda.Stream()
    # torch's first device allocation runs start-up work on the GPU; let it finish
    # before the first form, so it overlaps no measured launch
    torch.zeros(1 << 20, device="cuda:0").sum().item()
    torch.cuda.synchronize()
    # about a third of a second of matrix products first: the device leaves its
    # idle clocks before any form is warmed up or timed
    x = torch.randn(4096, 4096, device="cuda:0")
    t_spin = time.perf_counter()
    while time.perf_counter() - t_spin < 0.3:
        x = torch.tanh(x @ x)
        torch.cuda.synchronize()
    del x
    forms = {}
    # the other form first: its steps bring the device to its running clocks, so
    # no early step of the headline form pays for the ramp (a replay of 17-49 ms
    # instead of 12 ms was seen among the first timed steps of the form run first)
    order = ("fp32", "fp64") if args.headline == "fp64" else ("fp64", "fp32")
    for prec in order:
        print(f"bench: {w.name} {prec} warmup {args.warmup} steps {args.steps}", file=sys.stderr,
              flush=True)
        forms[prec] = run_form(bfi, torch, ctx, lat, sv, w, prec, args.steps, args.warmup, stream)
    host_path = host_path_leg(bfi, ctx, lat, sv)
    averaged = None
    if not args.no_observable_leg:
        averaged = observable_leg(bfi, torch, ctx, w, sv, args.steps, args.warmup, stream)
    pairs = None
    if not args.no_antithetic_leg and w.nx * w.nt <= 32:
        pairs = antithetic_leg(bfi, torch, ctx, w, sv, args.steps, args.warmup, stream)
    sampler = None
    if not args.no_sampler_leg and w.nx * w.nt <= 32:
        print("bench: Gaussian-proposal and spherical samplers", file=sys.stderr, flush=True)
        sampler = sampler_leg(bfi, ctx, w)
    adaptive = None
    if args.adaptive_budget_log2 > 0:
        print(f"bench: adaptive 10x2, budget 2^{args.adaptive_budget_log2} per nu",
              file=sys.stderr, flush=True)
        adaptive = adaptive_leg(bfi, ctx, args.adaptive_budget_log2)
    adaptive_target = None
    if args.adaptive_target_budget_log2 > 0 and w.name == "burgers10x2":
        print(f"bench: adaptive 10x2 to target, averaged observable, budget "
              f"2^{args.adaptive_target_budget_log2} per nu", file=sys.stderr, flush=True)
        # the workload's 1e-3 target, holdout-confirmed, FP32 form; and 1e-2 (which
        # a holdout pass confirms within the budget) in both forms and two seeds,
        # for the time each form takes to the same confirmed error (the rounds a
        # run needs depend on when a holdout check first passes: one seed per nu
        # measures that draw more than the forms)
        adaptive_target = adaptive_leg(bfi, ctx, args.adaptive_target_budget_log2,
                                       observables=("averaged",), forms=("fp32",),
                                       confirm=True, target=1e-3)
        adaptive_target += adaptive_leg(bfi, ctx, args.adaptive_target_budget_log2,
                                        observables=("averaged",), forms=("fp32", "fp64"),
                                        confirm=True, target=1e-2, seeds=(1, 2))
    adaptive_scale = None
    if args.adaptive_scale_budget_log2 > 0 and w.name == "burgers10x2":
        print(f"bench: adaptive scale run, budget 2^{args.adaptive_scale_budget_log2}",
              file=sys.stderr, flush=True)
        adaptive_scale = adaptive_scale_leg(bfi, ctx, args.adaptive_scale_budget_log2)
    if args.calibrate_copy_mib > 0:
        n = args.calibrate_copy_mib << 20
        x = torch.ones(n, dtype=torch.uint8, device="cuda:0")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    serving = None
    if args.serve_seconds > 0:
        print(f"bench: serving {args.serve_seconds:g} s at {args.serve_rate:g} req/s",
              file=sys.stderr, flush=True)
        serving = serve_leg(bfi, ctx, args.serve_seconds, args.serve_rate,
                            max_samples_per_thread=args.serve_max_samples_per_thread)
    bfi.bfi_context_destroy(ctx)

    head = forms[args.headline]
    r64, r32 = forms["fp64"]["result"], forms["fp32"]["result"]
    c0 = abs(r64["C"][0])
    dev = {"Z_rel": abs(r32["Z"] - r64["Z"]) / r64["Z"],
           "C_rel_max": float(np.max(np.abs(r32["C"] - r64["C"])) / c0)}
    stat = float(np.max(r64["C_err"]) / c0)

    slots = valu_slots_per_eval(w.nx, w.nt, args.headline)
    evals_per_launch = head["evals_per_step"]
    achieved = slots * evals_per_launch / (head["kernel_ms"] * 1e-3)
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_SLOTS / 1e12,
                "unit": "T FP64-rate lane slots/s", "frac": achieved / PEAK_SLOTS,
                "traffic": measured_traffic(w.name, args.headline),
                "kernel": f"mc_kernel {w.nx}x{w.nt} {args.headline} (graph replay: queue reset, "
                          "kernel, merge, record copy; HIP events on the launch stream)",
                "slots_per_eval": slots,
                "kernel_ms": head["kernel_ms"],
                "fp64_flops_per_eval": fp64_flops_per_eval(w.nx, w.nt),
                "fp64_flop_frac": (fp64_flops_per_eval(w.nx, w.nt) * evals_per_launch /
                                   (forms["fp64"]["kernel_ms"] * 1e-3)) / PEAK_FP64}
    line = {
        "metric": METRIC,
        "value": head["evals_per_s"],
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.headline == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "lattice": f"{w.nx}x{w.nt}", "nu": w.nu, "D": w.D,
                   "box": [-w.box, w.box], "subvolumes": w.n_sub, "evals_per_step": w.budget,
                   "seed": w.seed, "form": args.headline, "launch": head["launch"],
                   "work_items": head["n_items"]},
        "forms": {p: {"evals_per_s": f["evals_per_s"], "ms_per_step": f["ms_per_step"],
                      "step_ms_median": f["step_ms_median"], "step_ms_max": f["step_ms_max"],
                      "step_ms_each": f["step_ms_each"], "kernel_ms_each": f["kernel_ms_each"],
                      "kernel_ms": f["kernel_ms"], "kernel_ms_median": f["kernel_ms_median"],
                      "kernel_evals_per_s":
                          f["evals_per_step"] / (f["kernel_ms"] * 1e-3),
                      "valu_frac": valu_slots_per_eval(w.nx, w.nt, p) * f["evals_per_step"] /
                          (f["kernel_ms"] * 1e-3) / PEAK_SLOTS,
                      "launch": f["launch"]}
                  for p, f in forms.items()},
        "fp32_speedup_vs_fp64": forms["fp32"]["evals_per_s"] / forms["fp64"]["evals_per_s"],
        "fp32_deviation_vs_fp64": dev,
        "estimate": {"Z": r64["Z"], "log_Z": r64["log_Z"], "C": [float(c) for c in r64["C"]],
                     "max_rel_err_C": stat, "ess": r64["ess"]},
        "roofline": roofline,
        "host_path_pcie_inclusive": host_path,
    }
    if averaged is not None:
        rate = averaged["forms"][args.headline]["evals_per_s"] / head["evals_per_s"]
        ratio = np.asarray(averaged["paper_range"]["C_err_ratio"])
        averaged["equal_error_speedup"] = {"min_r": float(np.min(ratio ** 2) * rate),
                                           "median_r": float(np.median(ratio ** 2) * rate)}
        line["observable_averaged"] = averaged
    if pairs is not None:
        rate = pairs["forms"][args.headline]["evals_per_s"] / head["evals_per_s"]
        for b in pairs["error_at_equal_evals"]:
            b["equal_error_speedup_Z"] = b["Z_err_ratio"] ** 2 * rate
            b["equal_error_speedup_C_median_r"] = float(np.median(
                np.asarray(b["C_err_ratio"]) ** 2) * rate)
        pairs["rate_vs_single"] = rate
        line["antithetic_pairs"] = pairs
    if sampler is not None:
        line["sampler_gaussian_mixture"] = sampler
    if serving is not None:
        line["p99_latency_ms"] = serving["p99_ms"]
        line["serving"] = serving
    if adaptive is not None:
        line["adaptive"] = adaptive
    if adaptive_target is not None:
        line["adaptive_to_target"] = adaptive_target
        # time to the same holdout-confirmed error in both forms: FP64 seconds /
        # FP32 seconds over every (nu, seed) that both forms confirmed, in total
        # and per run
        speedup = {}
        for target in sorted({a["target"] for a in adaptive_target}):
            secs = {(a["form"], a["nu"], a["seed"]): a["seconds"] for a in adaptive_target
                    if a["target"] == target and a["status"] == "BFI_OK" and a.get("holdout_used")}
            both = sorted((nu, sd) for (form, nu, sd) in secs
                          if form == "fp32" and ("fp64", nu, sd) in secs)
            if both:
                t32 = sum(secs[("fp32", nu, sd)] for nu, sd in both)
                t64 = sum(secs[("fp64", nu, sd)] for nu, sd in both)
                speedup[f"{target:g}"] = {
                    "total": t64 / t32, "runs": len(both),
                    "per_run": {f"nu={nu} seed={sd}": secs[("fp64", nu, sd)] / secs[("fp32", nu, sd)]
                                for nu, sd in both}}
        line["fp32_speedup_at_target"] = speedup or None
    if adaptive_scale is not None:
        line["adaptive_scale"] = adaptive_scale
    if not args.no_cpu_baseline:
        print("bench: oracle CPU baseline", file=sys.stderr, flush=True)
        base, sub, rec = cpu_baseline(w, sv, args.cpu_samples_log2)
        line["cpu_baseline"] = base
        ctx = bfi.bfi_context_create(0)
        if os.path.exists(args.tune_cache):
            bfi.bfi_tune_load(ctx, args.tune_cache)
        line["error_vs_oracle"] = error_vs_oracle(bfi, ctx, w, sub, rec)
        bfi.bfi_context_destroy(ctx)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
