#!/usr/bin/env python
"""Throughput of the fused relaxed-CNF descent step on one MI355X.

A timed step is one pass of the whole hot path over the restart batch:
clause products and loss, the gathered gradient with the fused projected
update, and the exact unsat count of round(x) for every restart (all inside
galsat_step, with per-step loss and unsat traces); the K timed steps end
with the hand-off (galsat_round_check: ballot/popcount count, best restart
per formula and its assignment).  The state lives in HBM before the timed
region starts.

Prints ONE JSON line.  `value` = literal-evaluations per second
(R * L * K / time), `roofline` = the dominant kernel's algorithmic bytes per
launch over its event-timed average duration against the 8 TB/s HBM peak,
`cpu_baseline` = the FP64 oracle on a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "fwd+bwd literal-evals/s & % HBM peak; batched vs plain, 1e-5 rel vs FP64"
# the sources that define the variable pass (its traffic figure is only
# reported while these are unchanged since the counters were taken): the
# device helpers, the pass itself and its argument struct
CSRC = os.path.join(ROOT, "paper_2603_28796_amd", "csrc")
KERNEL_SRC = [os.path.join(CSRC, f) for f in ("galsat_device.h", "galsat_varpass.hip")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for path in KERNEL_SRC:
        with open(path, "rb") as fh:
            h.update(fh.read())
    text = open(os.path.join(CSRC, "galsat_internal.h")).read()
    start = text.index("struct VarPassArgs {")
    h.update(text[start:text.index("};", start)].encode())
    return h.hexdigest()[:16]


def read_traffic(workload: str, kernel: str):
    """Measured HBM bytes per launch from the committed counter summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.txt")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_hash = re.search(r"kernel_source_sha256_16:\s*(\w+)", text)
    m_bytes = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m_hash or not m_bytes or m_hash.group(1) != kernel_source_hash():
        return None
    return float(m_bytes.group(1))


def algorithmic_bytes(cnf, R, info, optimizer):
    """Compulsory bytes the variable pass must move per launch: the
    variable-major CSR, the clause-major CSR of the clauses it recomputes,
    the stored partial rows it reads, x read once and the next x written
    once (+ Adam moments read and written)."""
    n, m, L = cnf.n, cnf.m, cnf.L
    stored = int(info["stored_lits"])
    krec = int(info["recompute_max_len"])
    import numpy as np
    lens = np.diff(cnf.clause_ptr)
    rec = lens <= krec
    m_rec, L_rec = int(rec.sum()), int(lens[rec].sum())
    b = 4 * (n + 1) + 4 * L + 4 * (m_rec + 1) + 4 * L_rec + 8 * n * R + 4 * R * stored
    if optimizer == "adam":
        b += 16 * n * R
    return b


def stream_copy_gbps(nbytes: int = 2 << 30, reps: int = 5) -> float:
    """Device-to-device copy bandwidth on this GPU (bytes read + written per
    second), the measured counterpart of the HBM peak."""
    import torch

    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbps = 2.0 * nbytes * reps / (e0.elapsed_time(e1) / 1e3) / 1e9
    del a, b
    return gbps


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cnf, R, lr, budget_s: float):
    """The FP64 oracle's full step (gradient, unsat count, update) on the same
    instance, all restarts, repeated until about budget_s seconds."""
    import numpy as np
    import oracle

    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    x = np.random.default_rng(0).random((R, cnf.n))
    steps, t = 0, 0.0
    while t < budget_s and steps < 20:
        t0 = time.perf_counter()
        _, _, _, x = oracle.full_step(cnf, x, lr)
        t += time.perf_counter() - t0
        steps += 1
    v = R * cnf.L * steps / t
    return {"value": v, "unit": "literal-evals/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "sample": f"{steps} full FP64 steps (all {R} restarts) of the same instance, "
                      f"{t:.1f} s", "seconds": round(t, 2)}


def batched_vs_plain(steps: int):
    """The uneven batch of 4,096 formulas (R=32): every formula in each launch
    (the batched schedule, replayed from a captured graph) against one formula
    at a time with a launch per pass per step and no graph, same kernels,
    same steps, both from the same initial state in HBM."""
    import torch

    from paper_2603_28796_amd import inputs as I
    from paper_2603_28796_amd.galsat import Problem

    w = I.WORKLOADS["batch4096"]
    t0 = time.perf_counter()
    cnf = w.make()
    log(f"[bench] batch workload: F={cnf.F} n={cnf.n} L={cnf.L} "
        f"(generated in {time.perf_counter() - t0:.1f} s)")
    R = w.restarts
    out = {"workload": w.key, "formulas": cnf.F, "restarts": R, "steps": steps}
    x0 = None
    for name, sched, graph in (("batched", "general", True), ("plain", "plain", False)):
        prob = Problem(cnf, R, lr=w.lr, schedule=sched, use_graph=graph)
        if x0 is None:
            x0 = prob.init_state(I.SEED_BASE + 4)
        x = x0.clone()
        lt = torch.empty((steps, cnf.F, R), dtype=torch.float32, device="cuda")
        ut = torch.empty((steps, cnf.F, R), dtype=torch.int32, device="cuda")
        prob.step(x, 1, loss_trace=lt[:1], unsat_trace=ut[:1], trace=True)  # warm-up
        torch.cuda.synchronize()
        log(f"[bench] {name}: warm-up step done")
        x = x0.clone()
        if graph:
            prob.prepare(x, steps, loss_trace=lt, unsat_trace=ut)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        prob.step(x, steps, loss_trace=lt, unsat_trace=ut, trace=True)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        out[f"{name}_ms_per_step"] = ms / steps
        out[f"{name}_lit_evals_per_s"] = R * cnf.L * steps / (ms / 1e3)
        log(f"[bench] {name}: {ms / steps:.3f} ms/step")
        prob.close()
    out["speedup"] = out["plain_ms_per_step"] / out["batched_ms_per_step"]
    return out


def gumbel_and_handoff(cnf, R, steps: int):
    """The paper's own optimizer loop on the same instance (straight-through
    Gumbel-softmax, Adam lr 0.5, tau 1), then the hand-off to the CPU stage:
    100 candidates (Eq. 8), the top 0.05 % confident variables of each as
    unit literals (Eq. 9-10) and the 7 least confident of the selected
    restart as branching variables (Lemma 1).  Event-timed on the current
    stream, inputs resident in HBM."""
    import torch

    from paper_2603_28796_amd import inputs as I
    from paper_2603_28796_amd.galsat import Problem

    prob = Problem(cnf, R, optimizer="adam", lr=0.5)
    x0 = prob.init_state(I.SEED_BASE + 6)
    d = (x0 * 2.0 - 1.0).contiguous()  # initial logit differences in [-1, 1)
    opt = prob.new_opt_state(d)
    prob.gumbel_step(d, 2, opt_state=opt, seed=7, step0=0)  # warm-up
    e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    torch.cuda.synchronize()
    e[0].record()
    lt, ut = prob.gumbel_step(d, steps, opt_state=opt, seed=7, step0=2, trace=True)
    e[1].record()
    best = ut[-1].to(torch.int64).argmin(dim=1).to(torch.int32)  # fewest unsat, first index
    e[2].record()
    assign, conf = prob.candidates(d, best, num=100, seed=8, tau=1.0)
    off_u, units = prob.select_vars(conf, highest=True, frac=0.0005, min_count=1)
    conf1 = prob.confidence(d, best, tau=1.0)
    off_b, branch = prob.select_vars(conf1, highest=False, frac=0.0, min_count=7)
    e[3].record()
    torch.cuda.synchronize()
    ms = e[0].elapsed_time(e[1])
    out = {"optimizer": "adam", "lr": 0.5, "tau": 1.0, "steps": steps, "restarts": R,
           "ms_per_step": ms / steps, "lit_evals_per_s": R * cnf.L * steps / (ms / 1e3),
           "min_unsat_first_step": int(ut[0].min()), "min_unsat_last_step": int(ut[-1].min()),
           "handoff": {"candidates": 100, "ms": e[2].elapsed_time(e[3]),
                       "unit_literals_per_candidate": int(off_u[-1]),
                       "branching_vars": int(off_b[-1])}}
    prob.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="planted3sat_n1e5")
    ap.add_argument("--partials", default=None, help="auto | store | recompute")
    ap.add_argument("--plan", default=None, help="plan override, e.g. lpi=64,rpl=4")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="skip the event-timed kernel run")
    ap.add_argument("--graph", type=int, default=1, help="replay the step loop from a hipGraph")
    ap.add_argument("--schedule", default="auto", help="auto | general | lds | plain")
    ap.add_argument("--batch-steps", type=int, default=20,
                    help="steps of the batched vs one-formula-at-a-time comparison (0: skip)")
    ap.add_argument("--gumbel-steps", type=int, default=50,
                    help="steps of the straight-through Gumbel loop + hand-off timing (0: skip)")
    ap.add_argument("--tseitin", type=int, default=0,
                    help="run the workload after chain normalization to this clause width "
                         "(Eq. 6-7); also reports the unsat count on the original clauses")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build runs the hot path on a single MI355X "
              "(restart or formula sharding across GPUs is a design note, not implemented).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2603_28796_amd import inputs as I
    from paper_2603_28796_amd.galsat import Problem

    w = I.WORKLOADS[args.workload]
    t0 = time.perf_counter()
    cnf = w.make()
    original = None
    if args.tseitin:
        from paper_2603_28796_amd.galsat import tseitin
        original = cnf
        cnf = tseitin(cnf, args.tseitin)
        log(f"[bench] width-{args.tseitin} normalization: n {original.n} -> {cnf.n}, "
            f"m {original.m} -> {cnf.m}, L {original.L} -> {cnf.L}")
    log(f"[bench] workload {w.key}: n={cnf.n} m={cnf.m} L={cnf.L} F={cnf.F} R={w.restarts} "
        f"(generated in {time.perf_counter() - t0:.1f} s)")
    R = w.restarts
    partials = args.partials or {0: "auto", 1: "store", 2: "recompute"}[w.recompute]
    torch.cuda.set_device(0)
    prob = Problem(cnf, R, lr=w.lr, partials=partials, plan_override=args.plan,
                   use_graph=bool(args.graph), schedule=args.schedule)
    info = prob.info()
    log(f"[bench] plan: {info}")
    x = prob.init_state(I.SEED_BASE + 2)
    K, W = args.steps, args.warmup
    FR = cnf.F * R
    lt = torch.empty((max(K, W), cnf.F, R), dtype=torch.float32, device="cuda")
    ut = torch.empty((max(K, W), cnf.F, R), dtype=torch.int32, device="cuda")

    if W > 0:
        prob.step(x, W, loss_trace=lt[:W], unsat_trace=ut[:W], trace=True)
        prob.round_check(x)
    if args.graph:
        prob.prepare(x, K, loss_trace=lt[:K], unsat_trace=ut[:K])  # capture outside the timing
    torch.cuda.synchronize()
    log(f"[bench] warmup {W} steps done")

    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    prob.step(x, K, loss_trace=lt[:K], unsat_trace=ut[:K], trace=True)
    unsat, best, assign = prob.round_check(x)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    value = R * cnf.L * K / (ms / 1e3)
    log(f"[bench] timed {K} steps: {ms:.2f} ms ({ms / K:.4f} ms/step), {value:.4e} lit-evals/s; "
        f"min unsat {int(unsat.min())}, final mean loss {float(lt[K - 1].mean()):.3f}")
    normalized = None
    if original is not None:
        # the original variables keep their ids: round them and count the
        # original clauses they leave unsatisfied
        orig_prob = Problem(original, R, lr=w.lr)
        u0, _, _ = orig_prob.round_check(x[:original.n])
        torch.cuda.synchronize()
        normalized = {"width": args.tseitin, "original_n": original.n, "original_m": original.m,
                      "original_L": original.L, "min_unsat_original": int(u0.min()),
                      "min_unsat_normalized": int(unsat.min()),
                      "original_lit_evals_per_s": R * original.L * K / (ms / 1e3)}
        log(f"[bench] normalized run: {normalized}")
        orig_prob.close()

    roofline = None
    kernels = None
    if not args.no_profile:
        prob.profile(True)
        prob.step(x, K, loss_trace=lt[:K], unsat_trace=ut[:K], trace=True)
        prob.round_check(x)
        torch.cuda.synchronize()
        kernels = prob.kernel_times()
        prob.profile(False)
        log(f"[bench] kernel times: {kernels}")
        launches, tot = kernels.get("var_pass", (0, 0.0))
        # the LDS schedule runs every step in one launch with the state held
        # in LDS between steps: no per-step HBM roofline applies to it
        if launches and info["schedule"] != "lds":
            # the pass may be split into several launches per step (restart
            # tile groups): each launch moves its share of the step's bytes
            per_step = launches / K
            avg_ms = tot / launches
            ab = algorithmic_bytes(cnf, R, info, "sgd") / per_step
            achieved = ab / (avg_ms / 1e3) / 1e9
            traffic = read_traffic(w.key, "var_pass")
            copy = stream_copy_gbps()
            roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                        "traffic": traffic, "kernel": "k_var_pass",
                        "algorithmic_bytes_per_launch": ab, "avg_launch_ms": round(avg_ms, 5),
                        "launches_per_step": per_step,
                        # measured traffic rate and a measured copy on the same GPU
                        "traffic_GBps": round(traffic / (avg_ms / 1e3) / 1e9, 1) if traffic else None,
                        "stream_copy_GBps": round(copy, 1)}

    gumbel = None
    if args.gumbel_steps > 0 and not args.tseitin:
        prob.close()  # free the SGD handle's workspace first
        gumbel = gumbel_and_handoff(cnf, R, args.gumbel_steps)
        log(f"[bench] gumbel-ST + hand-off: {gumbel}")

    batch = None
    if args.batch_steps > 0:
        batch = batched_vs_plain(args.batch_steps)

    cpu = None
    if not args.no_cpu_baseline:
        log(f"[bench] cpu baseline (oracle, ~{args.cpu_seconds:.0f} s)")
        cpu = cpu_baseline(cnf, R, w.lr, args.cpu_seconds)
        log(f"[bench] cpu baseline: {cpu}")

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "literal-evals/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": ms / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.key + (f"/width{args.tseitin}" if args.tseitin else ""),
                   "description": w.description, "n": cnf.n, "m": cnf.m,
                   "L": cnf.L, "formulas": cnf.F, "restarts": R, "lr": w.lr, "partials": partials,
                   "schedule": info["schedule"], "lanes_per_item": info["lanes_per_item"],
                   **({"lds_restarts_per_group": info["lds_restarts_per_group"],
                       "lds_staged": info["lds_staged"]} if info["schedule"] == "lds" else {}),
                   "restarts_per_lane": info["restarts_per_lane"]},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "batched_vs_plain": batch,
        "normalized": normalized,
        "gumbel_st": gumbel,
        "kernel_ms": {k: {"launches": v[0], "avg_ms": round(v[1] / v[0], 5)}
                      for k, v in (kernels or {}).items()},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
