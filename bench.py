#!/usr/bin/env python3
"""Benchmark: softened-gravity accelerations/s at 4M particles, FP32C vs FP64.

Workload (precision study): 4,194,304 gas cells drawn as 512 Plummer clumps
(scale radii log-uniform in [1e-4, 0.05], 70% of the mass) on a uniform
background, softening = radius enclosing the 32 nearest neighbours, plus 2048
close sink binaries (separations 1e-5..1e-3, sink softening 1e-4), FP32 inputs,
seed 2.  One step = one full force evaluation on the GPU through the C ABI:
tree build (box, keys, radix sort, gather, topology, moments, groups), group
walk with quadrupole nodes at theta = 0.5, FP64 sink-sink sum, sink walk and
output scatter.  value = particles / step time (accelerations per second).

Reported beside it, on the same inputs:
  * the tree step in the plain FP32 and the FP64 forms;
  * the adjoint (accel_backward) against the force evaluation on one handle;
  * the direct (all-pairs) path in FP32C and FP64, one evaluation each;
  * the median and p99 relative force error of every form and path against
    the FP64 CPU oracle (direct sum) on a random target subsample;
  * the walk kernel's roofline (algorithmic FLOP per launch / launch time from
    HIP events on the library's stream), the direct kernel's likewise, the
    build's algorithmic HBM bytes per phase time, and the oracle itself timed
    on the host cores over the subsample.
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

# Algorithmic FLOP per interaction (FMA = 2, rsqrt = 1), counted from the
# evaluation code: particle pair 20, quadrupole node 54, monopole node 20.
FLOP_PP = 20
FLOP_PC = {0: 20, 2: 54}
PEAK_FP32_TFLOPS = 157.3          # MI355X vector FP32 (published, packed)
PEAK_FP32_NONPACKED_TFLOPS = 78.6
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
# Algorithmic HBM bytes per particle of the sort phase with FP32 inputs:
# box (read x 12) + keys (read x 12, write key 8 + index 4) + digit
# histograms (read keys 8) + 8 scatter passes (read and write key + index,
# 8 x 24) + gather (read index 4 and x, m, h 20, write 20) + sink positions
# (flags 8, scan 8, compaction 8).
SORT_BYTES_PER_PARTICLE = 12 + 24 + 8 + 8 * 24 + 44 + 24
# Files whose change invalidates the stored walk-kernel byte counters.
WALK_SOURCES = ("sf_internal.h", "sf_math.h", "sf_walk.h", "sf_walk.hip")
WALK_PMC_FILE = os.path.join(ROOT, "profiles", "walk_precision4m_pmc.md")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def walk_source_hash():
    h = hashlib.sha256()
    for f in WALK_SOURCES:
        with open(os.path.join(ROOT, "paper_2010_11254_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_walk_traffic():
    """HBM bytes per walk launch from the committed counter summary, if it was
    taken on the current walk sources (else None)."""
    try:
        with open(WALK_PMC_FILE) as fh:
            m = re.search(r"<!-- bench: (\{.*?\}) -->", fh.read())
    except OSError:
        return None
    if not m:
        return None
    rec = json.loads(m.group(1))
    if rec.get("src_sha") != walk_source_hash():
        return None
    return rec


def fractal_leg(np, torch, L, cpu_targets, cotangents, subsample):
    """Large run: fractal16m (16,777,216 gas in a 3-level Plummer-in-Plummer
    hierarchy + 10,000 sinks, seed 4), forward and backward at theta 0.5 and
    0.7, FP32C against FP64, with the force error on a random target sample."""
    from synth import fractal_cloud
    t0 = time.time()
    ps = fractal_cloud(1 << 24, 5000, 2500, seed=4)
    log(f"fractal16m: {ps.n} particles generated in {time.time() - t0:.1f}s")
    dev = torch.device("cuda", 0)
    x, m, h = (torch.as_tensor(v).to(dev) for v in (ps.x, ps.m, ps.h))
    ga, gp = cotangents(ps.n, seed=4, dtype=np.float32)
    ga, gp = torch.as_tensor(ga).to(dev), torch.as_tensor(gp).to(dev)
    acc = torch.empty((ps.n, 3), dtype=torch.float32, device=dev)
    pot = torch.empty((ps.n,), dtype=torch.float32, device=dev)
    sample = subsample(ps.n, cpu_targets, seed=4) if cpu_targets else None
    ref = None
    if sample is not None:
        from oracle import direct as odirect
        t0 = time.perf_counter()
        ref, _ = odirect.direct(ps.x.astype(np.float64), ps.m.astype(np.float64),
                                ps.h.astype(np.float64), targets=sample)
        log(f"fractal16m oracle: {sample.size} targets in {time.perf_counter() - t0:.1f}s")

    def ev_ms(fn, reps):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    out = {"n": ps.n, "n_gas": ps.n_gas, "n_sink": ps.n_sink, "seed": 4}
    for theta in (0.5, 0.7):
        for form in ("fp32c", "fp64"):
            o = L.make_opts(form=form, theta=theta, n_gas=ps.n_gas, collect_stats=True)

            def full():
                t = L.sf_grav_build_tree(x, m, h, o)
                L.sf_grav_accel(t, None, None, None, o, acc=acc, pot=pot)
                L.sf_grav_tree_free(t)
            o.collect_stats = 0
            step_ms = ev_ms(full, 3)
            o.collect_stats = 1
            t = L.sf_grav_build_tree(x, m, h, o)
            L.sf_grav_accel(t, None, None, None, o, acc=acc, pot=pot)
            torch.cuda.synchronize()
            r = {"step_ms": step_ms, "accels_per_s": ps.n / (step_ms * 1e-3)}
            if form == "fp32c":
                gf = L.sf_grav_tree_export(t, "group_first").numpy().astype(np.int64)
                gc = L.sf_grav_tree_export(t, "group_count").numpy().astype(np.int64)
                npc = L.sf_grav_tree_export(t, "group_npc").numpy().astype(np.int64)
                npp = L.sf_grav_tree_export(t, "group_npp").numpy().astype(np.int64)
                order = L.sf_grav_tree_export(t, "order").numpy()
                csum = np.concatenate([[0], np.cumsum(order < ps.n_gas)])
                active = csum[gf + gc] - csum[gf]
                r["n_pc"], r["n_pp"] = int((active * npc).sum()), int((active * npp).sum())
            o.collect_stats = 0
            r["accel_ms"] = ev_ms(lambda: L.sf_grav_accel(t, None, None, None, o, acc=acc,
                                                            pot=pot), 2)
            if ref is not None:
                got = acc[torch.as_tensor(sample, device=dev)].double().cpu().numpy()
                e = np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)
                r["rel_err"] = {"median": float(np.median(e)), "p99": float(np.quantile(e, 0.99))}
            r["backward_ms"] = ev_ms(lambda: L.sf_grav_accel_backward(t, None, None, None, o, ga,
                                                                      gp), 1)
            r["backward_over_accel"] = r["backward_ms"] / r["accel_ms"]
            L.sf_grav_tree_free(t)
            key = f"theta{theta}_{form}"
            out[key] = r
            log(f"fractal16m {key}: step {step_ms:.1f} ms, accel {r['accel_ms']:.1f} ms, "
                f"backward {r['backward_ms']:.1f} ms" +
                (f", p99 {r['rel_err']['p99']:.2e}" if "rel_err" in r else ""))
        fl = FLOP_PP * out[f"theta{theta}_fp32c"]["n_pp"] + FLOP_PC[2] * out[f"theta{theta}_fp32c"]["n_pc"]
        out[f"theta{theta}_fp32c"]["accel_tflops"] = fl / (out[f"theta{theta}_fp32c"]["accel_ms"] * 1e-3) / 1e12
        out[f"theta{theta}_fp32c_over_fp64"] = (out[f"theta{theta}_fp64"]["step_ms"] /
                                                out[f"theta{theta}_fp32c"]["step_ms"])
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--theta", type=float, default=0.5)
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target CPU time of the oracle baseline sample")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle leg (profiling runs)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 and plain-FP32 forms")
    ap.add_argument("--no-direct", action="store_true", help="skip the direct-path evaluations")
    ap.add_argument("--no-backward", action="store_true", help="skip the adjoint timing")
    ap.add_argument("--scale", type=float, default=1.0, help="particle-count scale (tests only)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run one 256 MiB elementwise copy first (calibrates HBM byte counters)")
    ap.add_argument("--fractal", action="store_true",
                    help="also run the 16M fractal workload (forward + backward, theta 0.5 and 0.7)")
    ap.add_argument("--leaf-cap", type=int, default=32)
    ap.add_argument("--group-cap", type=int, default=32)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported "
              "(how the walk would shard over GPUs is a design, not code)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2010_11254_amd import _lib as L
    from synth import cotangents, precision_cloud, subsample

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    n_gas = max(4096, int(round((1 << 22) * args.scale)))
    n_bin = max(16, int(round(2048 * args.scale)))
    t0 = time.time()
    ps = precision_cloud(n_gas, n_bin, seed=2)
    log(f"workload: {ps.n} particles ({ps.n_gas} gas, {ps.n_sink} sinks), "
        f"generated in {time.time() - t0:.1f}s")
    dev = torch.device("cuda", 0)
    x, m, h = (torch.as_tensor(v).to(dev) for v in (ps.x, ps.m, ps.h))
    if args.copy_probe:
        src = torch.empty(64 << 20, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.add(src, 1.0, out=dst)   # reads 256 MiB, writes 256 MiB
        torch.cuda.synchronize()
        del src, dst
    acc = torch.empty((ps.n, 3), dtype=torch.float32, device=dev)
    pot = torch.empty((ps.n,), dtype=torch.float32, device=dev)

    # oracle target sample: size it to the requested CPU time first
    sample = None
    xd = md = hd = None
    if not args.no_cpu:
        from oracle import direct as odirect
        xd, md, hd = (np.asarray(v, dtype=np.float64) for v in (ps.x, ps.m, ps.h))
        probe = subsample(ps.n, 256, seed=2)
        t0 = time.perf_counter()
        odirect.direct(xd, md, hd, targets=probe)
        rate = probe.size / (time.perf_counter() - t0)
        sample = subsample(ps.n, int(min(65536, max(512, rate * args.cpu_seconds))), seed=2)
    outs = {}

    def keep(name):
        if sample is not None:
            outs[name] = acc[torch.as_tensor(sample, device=dev)].double().cpu().numpy()

    def opts(form, timing=False, stats=False):
        return L.make_opts(form=form, theta=args.theta, order=2, leaf_cap=args.leaf_cap,
                           group_cap=args.group_cap, n_gas=ps.n_gas, timing=timing,
                           collect_stats=stats)

    def step(o):
        t = L.sf_grav_build_tree(x, m, h, o)
        L.sf_grav_accel(t, None, None, None, o, acc=acc, pot=pot)
        return t

    def timed(form, steps, warmup):
        o = opts(form, timing=True)
        for _ in range(warmup):
            L.sf_grav_tree_free(step(o))
        torch.cuda.synchronize()
        walk_ms, phase = [], {}
        t_start = time.perf_counter()
        for _ in range(steps):
            t = step(o)
            tm = L.sf_grav_get_timings(t)
            walk_ms.append(tm["walk"])
            for k, v in tm.items():
                if v is not None:
                    phase.setdefault(k, []).append(v)
            L.sf_grav_tree_free(t)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t_start) / steps
        return wall, float(np.mean(walk_ms)), {k: float(np.mean(v)) for k, v in phase.items()}

    def event_ms(fn, reps):
        """Mean time of fn() over reps calls, HIP events on the current stream
        (the one the library enqueues on)."""
        fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    # interaction counts of one evaluation (untimed), for the FLOP count
    t = step(opts("fp32c", stats=True))
    torch.cuda.synchronize()
    gf = L.sf_grav_tree_export(t, "group_first").numpy().astype(np.int64)
    gc = L.sf_grav_tree_export(t, "group_count").numpy().astype(np.int64)
    npc = L.sf_grav_tree_export(t, "group_npc").numpy().astype(np.int64)
    npp = L.sf_grav_tree_export(t, "group_npp").numpy().astype(np.int64)
    order = L.sf_grav_tree_export(t, "order").numpy()
    info = L.sf_grav_get_tree_info(t)
    L.sf_grav_tree_free(t)
    is_gas_sorted = (order < ps.n_gas).astype(np.int64)
    csum = np.concatenate([[0], np.cumsum(is_gas_sorted)])
    active = csum[gf + gc] - csum[gf]
    n_pc = int((active * npc).sum())
    n_pp = int((active * npp).sum())
    walk_flop = FLOP_PP * n_pp + FLOP_PC[2] * n_pc
    log(f"tree: {info['n_nodes']} nodes, {info['n_groups']} groups, max level {info['max_level']}; "
        f"interactions/target: {n_pc / ps.n_gas:.0f} node + {n_pp / ps.n_gas:.0f} particle")

    # headline: FP32C tree steps
    wall32, walk32, ph32 = timed("fp32c", args.steps, args.warmup)
    keep("tree_fp32c")
    log(f"fp32c: {wall32 * 1e3:.2f} ms/step, walk kernel {walk32:.2f} ms, phases "
        + ", ".join(f"{k} {v:.2f}" for k, v in ph32.items()))
    res = {}
    if not args.no_fp64:
        k64 = max(2, args.steps // 3)
        for form in ("fp64", "fp32"):
            wall, walk, ph = timed(form, k64, 1)
            keep("tree_" + form)
            res[form] = {"ms_per_step": wall * 1e3, "value": ps.n / wall, "walk_ms": walk,
                         "phases_ms": ph}
            log(f"{form}: {wall * 1e3:.2f} ms/step, walk kernel {walk:.2f} ms")

    # adjoint against the force evaluation on one handle (build excluded)
    adj = {}
    if not args.no_backward:
        ga, gp = cotangents(ps.n, seed=2, dtype=np.float32)
        ga, gp = torch.as_tensor(ga).to(dev), torch.as_tensor(gp).to(dev)
        for form in ("fp32c",) + (() if args.no_fp64 else ("fp64",)):
            o = opts(form)
            t = L.sf_grav_build_tree(x, m, h, o)
            fwd = event_ms(lambda: L.sf_grav_accel(t, None, None, None, o, acc=acc, pot=pot), 3)
            bwd = event_ms(lambda: L.sf_grav_accel_backward(t, None, None, None, o, ga, gp), 2)
            L.sf_grav_tree_free(t)
            build = res.get(form, {}).get("phases_ms") if form != "fp32c" else ph32
            b_ms = sum(build[k] for k in ("sort", "topology", "moments", "groups")) if build else None
            adj[form] = {"accel_ms": fwd, "backward_ms": bwd, "backward_over_accel": bwd / fwd}
            if b_ms is not None:
                adj[form]["with_build"] = (bwd + b_ms) / (fwd + b_ms)
            log(f"adjoint {form}: accel {fwd:.2f} ms, backward {bwd:.2f} ms, ratio {bwd / fwd:.2f}")
        del ga, gp

    # the same ratio on the differentiation workload (2^18 clustered gas,
    # per-particle h, seed 7; cotangents N(0, 1)); the build is timed with
    # events too, for the ratio that includes it
    adj_diff = {}
    if not args.no_backward:
        from synth import differentiation_cloud
        dcl = differentiation_cloud(1 << 18, seed=7)
        dx, dm, dh = (torch.as_tensor(v).to(dev) for v in (dcl.x, dcl.m, dcl.h))
        dga, dgp = cotangents(dcl.n, seed=7, dtype=np.float32)
        dga, dgp = torch.as_tensor(dga).to(dev), torch.as_tensor(dgp).to(dev)
        dacc = torch.empty((dcl.n, 3), dtype=torch.float32, device=dev)
        dpot = torch.empty(dcl.n, dtype=torch.float32, device=dev)
        for form in ("fp32c",) + (() if args.no_fp64 else ("fp64",)):
            o = L.make_opts(form=form, theta=args.theta, order=2, leaf_cap=args.leaf_cap,
                            group_cap=args.group_cap, n_gas=dcl.n_gas)
            bld = event_ms(lambda: L.sf_grav_tree_free(L.sf_grav_build_tree(dx, dm, dh, o)), 5)
            t = L.sf_grav_build_tree(dx, dm, dh, o)
            fwd = event_ms(lambda: L.sf_grav_accel(t, None, None, None, o, acc=dacc, pot=dpot), 10)
            bwd = event_ms(lambda: L.sf_grav_accel_backward(t, None, None, None, o, dga, dgp), 5)
            L.sf_grav_tree_free(t)
            adj_diff[form] = {"build_ms": bld, "accel_ms": fwd, "backward_ms": bwd,
                              "backward_over_accel": bwd / fwd,
                              "with_build": (bwd + bld) / (fwd + bld)}
            log(f"diff256k adjoint {form}: build {bld:.2f} ms, accel {fwd:.2f} ms, backward "
                f"{bwd:.2f} ms, ratio {bwd / fwd:.2f} ({(bwd + bld) / (fwd + bld):.2f} with the build)")
        del dx, dm, dh, dga, dgp, dacc, dpot

    # direct path: one evaluation per form over all pairs
    direct = {}
    if not args.no_direct:
        pairs = ps.n_gas * ps.n + ps.n_sink * ps.n_gas
        for form in ("fp32c", "fp64"):
            o = opts(form)
            k = min(ps.n, 65536)
            wx, wm, wh = x[:k].contiguous(), m[:k].contiguous(), h[:k].contiguous()
            L.sf_grav_accel(None, wx, wm, wh, L.make_opts(form=form, n_gas=min(k, ps.n_gas)),
                            acc=acc[:k], pot=pot[:k])   # loads the kernels
            torch.cuda.synchronize()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            L.sf_grav_accel(None, x, m, h, o, acc=acc, pot=pot)
            b.record()
            torch.cuda.synchronize()
            ms = a.elapsed_time(b)
            keep("direct_" + form)
            tf = FLOP_PP * pairs / (ms * 1e-3) / 1e12
            peak = PEAK_FP32_TFLOPS if form == "fp32c" else PEAK_FP64_TFLOPS
            direct[form] = {"ms": ms, "value": ps.n / (ms * 1e-3), "pairs_per_s": pairs / (ms * 1e-3),
                            "achieved_tflops": tf, "peak": peak, "frac": tf / peak}
            if form == "fp32c":
                direct[form]["frac_nonpacked"] = tf / PEAK_FP32_NONPACKED_TFLOPS
            log(f"direct {form}: {ms:.1f} ms, {pairs / (ms * 1e-3):.3e} pairs/s, {tf:.1f} TFLOP/s")

    cpu = None
    errs = {}
    if sample is not None:
        from oracle import direct as odirect
        t0 = time.perf_counter()
        ar, _ = odirect.direct(xd, md, hd, targets=sample)
        tcpu = time.perf_counter() - t0
        cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        cpu = {"value": sample.size / tcpu, "unit": "accels/s", "cores": cores, "kind": "oracle",
               "sample": f"{sample.size} random targets x all {ps.n} sources, FP64 direct sum, "
                         f"{tcpu:.1f}s"}
        log(f"oracle: {sample.size} targets in {tcpu:.1f}s on {cores} threads")
        nref = np.linalg.norm(ar, axis=1)
        ok = nref > 0
        for name, out in outs.items():
            e = np.linalg.norm(out - ar, axis=1)[ok] / nref[ok]
            errs[name] = {"median": float(np.median(e)), "p99": float(np.quantile(e, 0.99))}
            log(f"error {name}: median {errs[name]['median']:.3e}, p99 {errs[name]['p99']:.3e}")

    achieved = walk_flop / (walk32 * 1e-3) / 1e12
    traffic = None
    pmc = stored_walk_traffic()
    if pmc is not None:
        traffic = pmc["bytes_per_launch"]
    sort_ms = ph32.get("sort")
    line = {
        "metric": "softened-gravity accels/sec at 4M particles (FP32c vs FP64); p99 force err",
        "value": ps.n / wall32,
        "unit": "accels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall32 * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "precision4m: 4,194,304 clustered gas + 2048 sink binaries",
                   "n": ps.n, "n_gas": ps.n_gas, "n_sink": ps.n_sink, "inputs": "fp32",
                   "path": "tree", "theta": args.theta, "order": "quadrupole",
                   "form": "fp32c", "leaf_cap": args.leaf_cap, "group_cap": args.group_cap,
                   "seed": 2},
        "roofline": {"bound": "alu", "kernel": "k_walk_groups", "achieved": achieved,
                     "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS,
                     "frac_nonpacked": achieved / PEAK_FP32_NONPACKED_TFLOPS,
                     "traffic": traffic,
                     "walk_ms": walk32, "flop_per_launch": walk_flop,
                     "interactions_per_s": (n_pc + n_pp) / (walk32 * 1e-3),
                     "n_pc": n_pc, "n_pp": n_pp},
        "cpu_baseline": cpu,
        "phases_ms": ph32,
    }
    if sort_ms:
        gbs = SORT_BYTES_PER_PARTICLE * ps.n / (sort_ms * 1e-3) / 1e9
        line["build_sort_hbm"] = {"bytes_per_particle": SORT_BYTES_PER_PARTICLE,
                                  "achieved_gbs": gbs, "frac": gbs / PEAK_HBM_GBS}
    for form in ("fp64", "fp32"):
        if form in res:
            line[form] = res[form]
    if "fp64" in res:
        line["fp32c_over_fp64"] = res["fp64"]["ms_per_step"] / (wall32 * 1e3)
    if adj:
        line["adjoint"] = adj
    if adj_diff:
        line["adjoint_diff256k"] = adj_diff
    if direct:
        line["direct"] = direct
        if "fp64" in direct:
            line["direct"]["fp32c_over_fp64"] = direct["fp64"]["ms"] / direct["fp32c"]["ms"]
    if errs:
        line["rel_err"] = errs
        if "tree_fp32c" in errs:
            line["rel_err_fp32c"] = errs["tree_fp32c"]
    if args.fractal:
        del x, m, h, acc, pot
        torch.cuda.empty_cache()
        line["fractal16m"] = fractal_leg(np, torch, L, 0 if args.no_cpu else 2048, cotangents,
                                         subsample)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
