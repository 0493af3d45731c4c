#!/usr/bin/env python3
"""Benchmark: softened-gravity accelerations/s at 4M particles, FP32C vs FP64,
with the p99 relative force error against the FP64 CPU oracle.

Headline workload (precision study, precision4m): 4,194,304 gas cells drawn
as 512 Plummer clumps (scale radii log-uniform in [1e-4, 0.05], 70% of the
mass) on a uniform background, softening = radius enclosing the 32 nearest
neighbours, plus 2048 close sink binaries (separations 1e-5..1e-3, sink
softening 1e-4), FP32 inputs, seed 2.  One step = one full force evaluation
through the C ABI: tree build (box, keys, radix sort, gather, topology,
moments, groups), the previous step's field handed to the tree (for the
acceleration-based opening criterion), group walk with quadrupole nodes at
theta = 0.5 combined with the relative criterion (alpha = 0.003), FP64
sink-sink sum, sink walk and output scatter.  value = particles / step time.

Reported beside it:
  * the same step without the relative criterion (theta only), and in the
    FP64 and plain FP32 forms (FP32C/FP64 ratio at equal accuracy);
  * the adjoint against the force evaluation on one handle (precision4m,
    diff256k, fractal16m);
  * the direct path in FP32C, plain FP32 and FP64, one evaluation each;
  * the other evaluations on a precision4m handle: tidal tensor and jerk
    (with their error on an oracle sample), the symmetrised adaptive gas
    softening, the 6-bin columns and IR energy density, and the sinks-only
    pass and Hermite step on the 4096 sinks;
  * uniform4k (4096 particles, FP64, monopole) and clustered1m (2^20 gas +
    256 sinks) tree errors and times; fractal16m (2^24 gas + 10^4 sinks)
    forward and backward at theta 0.5 and 0.7;
  * median and p99 relative force error of every leg against the oracle on
    random target samples (65,536 at precision4m), computed by a background
    process running the oracle on the host cores while the GPU legs run;
  * the walk kernel's roofline (algorithmic FLOP per launch / launch time
    from HIP events on the library's stream), the direct kernel's and the
    build's, and the oracle's own throughput (cpu_baseline).
"""
import argparse
import hashlib
import json
import os
import re
import subprocess
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic FLOP per interaction (FMA = 2, rsqrt = 1), counted from the
# evaluation code: particle pair 20, quadrupole node 54, monopole node 20.
FLOP_PP = 20
FLOP_PC = {0: 20, 2: 54}
# With the tidal tensor and jerk in the same walk: particle pair 63 (the
# pair's g and phi, T from F and F'/r, j from the relative velocity);
# quadrupole node 98 (its g and phi, 54, plus the monopole T and j terms,
# sharing r and 1/r with them).
FLOP_PP_TIDAL = 63
FLOP_PC_TIDAL = 98
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
# Algorithmic HBM bytes per particle of the walk: one pass over the sorted
# particles (x, m, h: 20), the node records (about 0.11 nodes per particle at
# 128 + 48 bytes: 20), the groups (2 per 21.7 particles: negligible) and the
# outputs (acc and pot: 16).
WALK_BYTES_PER_PARTICLE = 20 + 20 + 16
SIDE_PHASES = ("sinksink", "sinkwalk")   # timers of the library's second stream
# Relative (acceleration-based) opening criterion tolerances: quadrupole
# workloads, and the monopole uniform sphere.
ALPHA = 0.003
ALPHA_MONO = 0.0005
# Oracle target samples per workload (R18: 65,536 at precision4m), and the
# sample of the tidal tensor and jerk check at precision4m (its own seed).
SAMPLES = {"precision4m": 65536, "clustered1m": 8192, "fractal16m": 2048, "uniform4k": 4096}
TIDAL_SAMPLE, TIDAL_SEED = 2048, 22
# Targets of the sample whose oracle evaluation is timed as the CPU baseline
# (at precision4m about 25 s of FP64 direct sum on 14 host threads).
BASELINE_TARGETS = 16384
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


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads():
    return int(os.environ.get("OMP_NUM_THREADS", 0)) or len(os.sched_getaffinity(0))


# ---------------------------------------------------------------- oracle worker

def make_workload(name):
    from synth import make_config
    return make_config(name)


def oracle_worker(outdir, names):
    """Runs in its own process: regenerate each workload from its seed, draw
    its target sample and evaluate the FP64 oracle direct sum on it."""
    import numpy as np
    from oracle import direct as odirect
    from synth import subsample
    for name in names:
        t0 = time.time()
        ps = make_workload(name)
        tg = time.time() - t0
        sample = subsample(ps.n, SAMPLES[name], seed=_seed(name))
        x, m, h = (np.asarray(v, dtype=np.float64) for v in (ps.x, ps.m, ps.h))
        # the timed part is the sample's first BASELINE_TARGETS targets (tens
        # of seconds); the rest, needed only for the error check, is untimed
        nb = min(sample.size, BASELINE_TARGETS)
        t0 = time.perf_counter()
        ref, _ = odirect.direct(x, m, h, targets=sample[:nb])
        tc = time.perf_counter() - t0
        if nb < sample.size:
            rest, _ = odirect.direct(x, m, h, targets=sample[nb:])
            ref = np.concatenate([ref, rest])
        np.save(os.path.join(outdir, f"{name}_ref.npy"), ref)
        np.save(os.path.join(outdir, f"{name}_sample.npy"), sample)
        if name == "precision4m":   # tidal tensor and jerk on their own sample
            from synth import velocities
            ts = subsample(ps.n, TIDAL_SAMPLE, seed=TIDAL_SEED)
            v = velocities(ps.n, seed=_seed(name)).astype(np.float64)
            Tr, Jr = odirect.direct_tidal(x, m, h, v, targets=ts)
            np.save(os.path.join(outdir, "precision4m_tidal_T.npy"), Tr)
            np.save(os.path.join(outdir, "precision4m_tidal_J.npy"), Jr)
        with open(os.path.join(outdir, f"{name}.json"), "w") as fh:
            json.dump({"targets": int(nb), "sources": int(ps.n), "seconds": tc,
                       "gen_seconds": tg, "threads": host_threads()}, fh)
        print(f"[oracle] {name}: {sample.size} targets x {ps.n} sources, the first {nb} "
              f"timed: {tc:.1f}s", flush=True, file=sys.stderr)


def _seed(name):
    return {"uniform4k": 0, "clustered1m": 1, "precision4m": 2, "diff256k": 7, "fractal16m": 4}[name]


# ---------------------------------------------------------------- GPU helpers

class Gpu:
    def __init__(self, np, torch, L):
        self.np, self.torch, self.L = np, torch, L
        self.dev = torch.device("cuda", 0)

    def upload(self, ps):
        return [self.torch.as_tensor(v).to(self.dev) for v in (ps.x, ps.m, ps.h)]

    def event_ms(self, fn, reps):
        """Mean time of fn() over reps calls, HIP events on the current stream
        (the one the library enqueues on)."""
        torch = self.torch
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


class ClockSampler:
    """Samples the GPU's graphics clock with `amd-smi` in a background thread
    while a leg runs (a child process, started and waited for; None when the
    tool is missing).  The clock is recorded because the VALU peaks assume
    2.4 GHz.  Off in profiling runs (`--no-cpu`): a profiler preloads itself
    into child programs too, and `amd-smi` is a script whose interpreter is
    started by exec from such a child."""

    enabled = True

    def __init__(self):
        import threading
        self.mhz, self._stop = [], threading.Event()
        self._thread = threading.Thread(target=self._run, daemon=True)

    def _sample(self):
        import numpy as np
        try:
            out = subprocess.run(["amd-smi", "metric", "-c", "--json"], capture_output=True,
                                 text=True, timeout=10).stdout
            data = json.loads(out)
            gpus = data["gpu_data"] if isinstance(data, dict) else data
            clocks = gpus[0]["clock"]
            vals = [c["clk"]["value"] for k, c in clocks.items()
                    if k.startswith("gfx") and isinstance(c, dict) and isinstance(c.get("clk"), dict)
                    and isinstance(c["clk"].get("value"), (int, float))]
            return float(np.mean(vals)) if vals else None
        except Exception:   # no tool, no permission, other output: no sample
            return None

    def _run(self):
        while not self._stop.is_set():
            v = self._sample()
            if v is None:
                return
            self.mhz.append(v)

    def __enter__(self):
        if ClockSampler.enabled:
            self._thread.start()
        return self

    def __exit__(self, *exc):
        self._stop.set()
        if self._thread.is_alive():
            self._thread.join(timeout=15)

    def summary(self):
        import numpy as np
        if not self.mhz:
            return None
        return {"median": float(np.median(self.mhz)), "max": float(np.max(self.mhz)),
                "samples": len(self.mhz), "tool": "amd-smi metric -c (mean over gfx domains)"}


class TreeLeg:
    """Repeated tree steps on one workload: build, previous field (when the
    relative criterion is on), walk.  The field of step k is the output of
    step k - 1 (the first from a theta-only evaluation)."""

    def __init__(self, g, ps, x, m, h, form, theta, alpha, order=2, leaf_cap=32, group_cap=32):
        self.g, self.ps, self.x, self.m, self.h = g, ps, x, m, h
        L, torch = g.L, g.torch
        self.opts = dict(form=form, theta=theta, order=order, leaf_cap=leaf_cap,
                         group_cap=group_cap, n_gas=ps.n_gas, alpha=alpha)
        self.alpha = alpha
        n = ps.n
        self.acc = [torch.empty((n, 3), dtype=x.dtype, device=g.dev) for _ in range(2)]
        self.pot = torch.empty((n,), dtype=x.dtype, device=g.dev)
        self.cur = 0
        if alpha is not None:   # field of a theta-only evaluation to start from
            # (with statistics on: another kernel instance than the timed walks)
            o = L.make_opts(**{**self.opts, "alpha": None, "collect_stats": True})
            t = L.sf_grav_build_tree(x, m, h, o)
            L.sf_grav_accel(t, None, None, None, o, acc=self.acc[1], pot=self.pot)
            L.sf_grav_tree_free(t)

    def o(self, **kw):
        return self.g.L.make_opts(**{**self.opts, **kw})

    def step(self, o):
        L = self.g.L
        t = L.sf_grav_build_tree(self.x, self.m, self.h, o)
        if self.alpha is not None:
            L.sf_grav_tree_set_field(t, self.acc[1 - self.cur])
        L.sf_grav_accel(t, None, None, None, o, acc=self.acc[self.cur], pot=self.pot)
        self.cur = 1 - self.cur
        return t

    @property
    def last(self):
        return self.acc[1 - self.cur]

    def timed(self, steps, warmup):
        """Wall time per step (host clock around synchronised steps) and the
        mean per-phase HIP event times."""
        np, torch, L = self.g.np, self.g.torch, self.g.L
        o = self.o(timing=True)
        for _ in range(warmup):
            L.sf_grav_tree_free(self.step(o))
        torch.cuda.synchronize()
        phase, per_step = {}, []
        t0 = time.perf_counter()
        for _ in range(steps):
            s0 = time.perf_counter()
            t = self.step(o)
            for k, v in L.sf_grav_get_timings(t).items():   # synchronises the stream
                if v is not None:
                    phase.setdefault(k, []).append(v)
            per_step.append((time.perf_counter() - s0) * 1e3)
            L.sf_grav_tree_free(t)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / steps
        walk = phase.get("walk", [])
        # the sink-sink sum and the sink walk run on the library's second
        # stream beside the group walk: their event intervals include waiting
        # for execution slots that the walk holds, so they are kept apart
        # from the serial phases
        self.side_spans = {k: float(np.mean(phase.pop(k))) for k in SIDE_PHASES if k in phase}
        self.step_stats = {"ms_median": float(np.median(per_step)), "ms_min": float(np.min(per_step)),
                           "walk_ms_median": float(np.median(walk)) if walk else None,
                           "walk_ms_min": float(np.min(walk)) if walk else None}
        return wall, {k: float(np.mean(v)) for k, v in phase.items()}

    def stats(self):
        """Interaction totals of one (untimed) evaluation."""
        L = self.g.L
        t = self.step(self.o(collect_stats=True))
        st = L.sf_grav_get_stats(t)
        info = L.sf_grav_get_tree_info(t)
        L.sf_grav_tree_free(t)
        return st, info

    def handle(self):
        """A built tree with the field set, for accel/backward timings."""
        L = self.g.L
        o = self.o()
        t = L.sf_grav_build_tree(self.x, self.m, self.h, o)
        if self.alpha is not None:
            L.sf_grav_tree_set_field(t, self.last)
        return t, o


def errors(np, got, ref):
    nref = np.linalg.norm(ref, axis=1)
    ok = nref > 0
    e = np.linalg.norm(got - ref, axis=1)[ok] / nref[ok]
    return {"median": float(np.median(e)), "p99": float(np.quantile(e, 0.99)),
            "max": float(e.max()), "targets": int(ok.sum())}


# ---------------------------------------------------------------- main

def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--theta", type=float, default=0.5)
    ap.add_argument("--alpha", type=float, default=ALPHA,
                    help="relative opening criterion of the headline (negative: off)")
    ap.add_argument("--no-cpu", action="store_true",
                    help="skip the oracle and the clock sampler (profiling runs)")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the headline FP32C steps (profiling runs)")
    ap.add_argument("--no-fractal", action="store_true", help="skip the 16M fractal workload")
    ap.add_argument("--with-adjoint", action="store_true",
                    help="with --headline-only: one FP32C adjoint on a headline handle (profiling)")
    ap.add_argument("--with-direct", action="store_true",
                    help="with --headline-only: the direct path in each form (profiling)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run one 256 MiB elementwise copy first (calibrates HBM byte counters)")
    ap.add_argument("--leaf-cap", type=int, default=32)
    ap.add_argument("--group-cap", type=int, default=32)
    ap.add_argument("--oracle-worker", metavar="DIR", help=argparse.SUPPRESS)
    ap.add_argument("--oracle-names", default="", help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.oracle_worker:
        oracle_worker(args.oracle_worker, [s for s in args.oracle_names.split(",") if s])
        return
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported "
              "(how the walk would shard over GPUs is a design, not code)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2010_11254_amd import _lib as L
    from synth import cotangents, differentiation_cloud, subsample, velocities

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    alpha = args.alpha if args.alpha >= 0 else None
    ClockSampler.enabled = not args.no_cpu
    g = Gpu(np, torch, L)

    # the oracle runs beside the GPU legs, on all host threads but two
    worker, outdir = None, None
    names = ["precision4m", "uniform4k", "clustered1m"] + ([] if args.no_fractal else ["fractal16m"])
    if not (args.no_cpu or args.headline_only):
        outdir = tempfile.mkdtemp(prefix="sfgrav_oracle_")
        threads = max(1, host_threads() - 2)
        env = dict(os.environ, OMP_NUM_THREADS=str(threads))
        worker = subprocess.Popen([sys.executable, os.path.abspath(__file__), "--oracle-worker",
                                   outdir, "--oracle-names", ",".join(names)], env=env)
    samples = {n: subsample(make_workload_size(n), SAMPLES[n], seed=_seed(n)) for n in names}
    samples["precision4m_tidal"] = subsample(make_workload_size("precision4m"), TIDAL_SAMPLE,
                                             seed=TIDAL_SEED)
    kept = {}   # (workload, leg) -> outputs at the workload's sample

    def keep(name, leg, acc):
        kept[(name, leg)] = acc[torch.as_tensor(samples[name], device=g.dev)].double().cpu().numpy()

    t0 = time.time()
    ps = make_workload("precision4m")
    log(f"precision4m: {ps.n} particles ({ps.n_gas} gas, {ps.n_sink} sinks), "
        f"generated in {time.time() - t0:.1f}s")
    x, m, h = g.upload(ps)
    if args.copy_probe:
        src = torch.empty(64 << 20, dtype=torch.float32, device=g.dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.add(src, 1.0, out=dst)   # reads 256 MiB, writes 256 MiB
        torch.cuda.synchronize()
        del src, dst
    caps = dict(leaf_cap=args.leaf_cap, group_cap=args.group_cap)

    # headline: FP32C tree steps, theta + relative criterion
    head = TreeLeg(g, ps, x, m, h, "fp32c", args.theta, alpha, **caps)
    st, info = head.stats()
    n_pc, n_pp = st["n_pc"], st["n_pp"]
    walk_flop = FLOP_PP * n_pp + FLOP_PC[2] * n_pc
    log(f"tree: {info['n_nodes']} nodes, {info['n_groups']} groups, max level {info['max_level']}; "
        f"interactions/target: {n_pc / ps.n_gas:.0f} node + {n_pp / ps.n_gas:.0f} particle")
    wall32, ph32 = head.timed(args.steps, args.warmup)
    side32 = head.side_spans
    step_stats = head.step_stats
    keep("precision4m", "tree_fp32c", head.last)
    clocks = {}
    if not args.headline_only:
        # the graphics clock while headline steps run (untimed, about 3 s)
        with ClockSampler() as cs:
            t_end = time.time() + 3.0
            while time.time() < t_end:
                L.sf_grav_tree_free(head.step(head.o()))
            torch.cuda.synchronize()
        clocks["tree_steps"] = cs.summary()
    walk32 = ph32["walk"]
    log(f"fp32c: {wall32 * 1e3:.2f} ms/step, walk kernel {walk32:.2f} ms, phases "
        + ", ".join(f"{k} {v:.2f}" for k, v in ph32.items()))

    res, adj, direct, tidal, extra = {}, {}, {}, {}, {}
    if not args.headline_only:
        # theta only (no relative criterion), and the FP64 / plain FP32 forms
        k2 = max(2, args.steps // 3)
        legs = [("fp32c_theta_only", "fp32c", None)] + [(f, f, alpha) for f in ("fp64", "fp32")]
        for key, form, al in legs:
            leg = TreeLeg(g, ps, x, m, h, form, args.theta, al, **caps)
            wall, ph = leg.timed(k2, 1)
            keep("precision4m", "tree_" + key, leg.last)
            res[key] = {"ms_per_step": wall * 1e3, "value": ps.n / wall, "walk_ms": ph.get("walk"),
                        "phases_ms": ph, "alpha": al}
            if al is None and form == "fp32c":
                s2, _ = leg.stats()
                res[key].update(n_pc=s2["n_pc"], n_pp=s2["n_pp"])
            log(f"{key}: {wall * 1e3:.2f} ms/step, walk kernel {ph.get('walk', 0):.2f} ms")
            del leg

        # adjoint against the force evaluation on one handle (build excluded)
        ga, gp = (torch.as_tensor(v).to(g.dev) for v in cotangents(ps.n, seed=2, dtype=np.float32))
        for form in ("fp32c", "fp64"):
            leg = head if form == "fp32c" else TreeLeg(g, ps, x, m, h, form, args.theta, alpha, **caps)
            t, o = leg.handle()
            fwd = g.event_ms(lambda: L.sf_grav_accel(t, None, None, None, o, acc=leg.acc[0],
                                                     pot=leg.pot), 3)
            bwd = g.event_ms(lambda: L.sf_grav_accel_backward(t, None, None, None, o, ga, gp), 2)
            L.sf_grav_tree_free(t)
            adj[form] = {"accel_ms": fwd, "backward_ms": bwd, "backward_over_accel": bwd / fwd}
            log(f"adjoint {form}: accel {fwd:.2f} ms, backward {bwd:.2f} ms, ratio {bwd / fwd:.2f}")
        del ga, gp

        # tidal tensor and jerk in the same walk (Sec. 2.2), FP32C, same
        # criterion and field as the headline, against the force evaluation
        vel = torch.as_tensor(velocities(ps.n, seed=2)).to(g.dev)
        t, o = head.handle()
        fwd = g.event_ms(lambda: L.sf_grav_accel(t, None, None, None, o, acc=head.acc[0],
                                                 pot=head.pot), 3)
        tms = g.event_ms(lambda: L.sf_grav_accel_tidal(t, o, vel=vel), 3)
        _, _, tid, jerk = L.sf_grav_accel_tidal(t, o, vel=vel)
        L.sf_grav_tree_free(t)
        keep("precision4m_tidal", "T", tid)
        keep("precision4m_tidal", "j", jerk)
        # the same lists as the headline walk: its interaction totals apply
        tf = (FLOP_PP_TIDAL * n_pp + FLOP_PC_TIDAL * n_pc) / (tms * 1e-3) / 1e12
        tidal = {"accel_ms": fwd, "tidal_jerk_ms": tms, "ratio": tms / fwd, "form": "fp32c",
                 "alpha": alpha, "achieved_tflops": tf, "peak": PEAK_FP32_TFLOPS,
                 "frac": tf / PEAK_FP32_TFLOPS, "frac_nonpacked": tf / PEAK_FP32_NONPACKED_TFLOPS}
        log(f"tidal+jerk fp32c: {tms:.2f} ms against accel {fwd:.2f} ms ({tms / fwd:.2f}x), "
            f"{tf:.1f} TFLOP/s")
        del tid, jerk

        # the other tree-pass evaluations on the same handle (times only:
        # their parity is in the tests): symmetrised adaptive gas softening
        # (softening here is the 32-NN radius, not re-solved) and the
        # radiation sums (6-bin columns, IR energy density of the sinks)
        t, o = head.handle()
        lum = torch.zeros(ps.n, dtype=torch.float32, device=g.dev)
        lum[ps.n_gas:] = torch.exp(torch.randn(ps.n_sink, generator=torch.Generator().manual_seed(2))).to(g.dev)
        extra["adaptive_softening_ms"] = g.event_ms(lambda: L.sf_grav_accel_adaptive(t, o), 2)
        extra["rad_sums_ms"] = g.event_ms(lambda: L.sf_grav_rad_sums(t, o, lum=lum, c_light=1.0), 3)
        extra["accel_ms"] = fwd
        L.sf_grav_tree_free(t)
        log(f"adaptive softening {extra['adaptive_softening_ms']:.2f} ms, radiation sums "
            f"{extra['rad_sums_ms']:.2f} ms (accel {fwd:.2f} ms)")
        # sink dynamics on the workload's 4096 sinks (FP64): sinks-only pass
        # with time scales, and one modified Hermite step
        sl = slice(ps.n_gas, ps.n)
        sx, sm_, sh = (torch.as_tensor(np.ascontiguousarray(v[sl], dtype=np.float64)).to(g.dev)
                       for v in (ps.x, ps.m, ps.h))
        sv = vel[ps.n_gas:].double().contiguous()
        extra["sinks_pass_ms"] = g.event_ms(lambda: L.sf_grav_sinks(sx, sv, sm_, sh, eta=0.01), 5)
        extra["sink_hermite_step_ms"] = g.event_ms(
            lambda: L.sf_grav_sink_hermite(sx, sv, sm_, sh, 1e-9), 5)
        extra["n_sink"] = ps.n_sink
        log(f"sinks pass {extra['sinks_pass_ms']:.3f} ms, Hermite step "
            f"{extra['sink_hermite_step_ms']:.3f} ms ({ps.n_sink} sinks)")
        del vel, lum, sx, sm_, sh, sv

        direct = direct_leg(g, ps, x, m, h, head, keep, clocks)
    if args.headline_only and args.with_direct:
        direct = direct_leg(g, ps, x, m, h, head, keep, clocks)
    if args.headline_only and args.with_adjoint:
        ga, gp = (torch.as_tensor(v).to(g.dev) for v in cotangents(ps.n, seed=2, dtype=np.float32))
        t, o = head.handle()
        bwd = g.event_ms(lambda: L.sf_grav_accel_backward(t, None, None, None, o, ga, gp), 1)
        L.sf_grav_tree_free(t)
        adj["fp32c"] = {"backward_ms": bwd}
        log(f"adjoint fp32c: backward {bwd:.2f} ms")
    del x, m, h, head
    torch.cuda.empty_cache()

    others = {}
    if not args.headline_only:
        # uniform4k: FP64, monopole, theta 0.5 with and without the criterion
        u = make_workload("uniform4k")
        ux, um, uh = g.upload(u)
        others["uniform4k"] = {"n": u.n, "order": "monopole", "dtype": "fp64"}
        for key, al in (("theta_only", None), ("relative", ALPHA_MONO)):
            leg = TreeLeg(g, u, ux, um, uh, "fp64", args.theta, al, order=0, leaf_cap=16,
                          group_cap=64)
            wall, _ = leg.timed(5, 2)
            keep("uniform4k", key, leg.last)
            others["uniform4k"][key] = {"ms_per_step": wall * 1e3, "alpha": al}
        # clustered1m: FP32C, quadrupole
        c1 = make_workload("clustered1m")
        cx, cm, ch = g.upload(c1)
        others["clustered1m"] = {"n": c1.n, "n_sink": c1.n_sink, "order": "quadrupole",
                                 "form": "fp32c"}
        for key, al in (("theta_only", None), ("relative", alpha)):
            leg = TreeLeg(g, c1, cx, cm, ch, "fp32c", args.theta, al, **caps)
            wall, ph = leg.timed(args.steps, 2)
            s1, _ = leg.stats()
            keep("clustered1m", key, leg.last)
            others["clustered1m"][key] = {"ms_per_step": wall * 1e3, "value": c1.n / wall,
                                          "walk_ms": ph.get("walk"), "alpha": al,
                                          "n_pc": s1["n_pc"], "n_pp": s1["n_pp"]}
            log(f"clustered1m {key}: {wall * 1e3:.2f} ms/step")
        del cx, cm, ch, leg
        # diff256k: adjoint ratio (theta only, as the workload specifies)
        d = differentiation_cloud(1 << 18, seed=7)
        dx, dm, dh = g.upload(d)
        dga, dgp = (torch.as_tensor(v).to(g.dev) for v in cotangents(d.n, seed=7, dtype=np.float32))
        others["diff256k"] = {}
        for form in ("fp32c", "fp64"):
            o = L.make_opts(form=form, theta=args.theta, n_gas=d.n_gas, **caps)
            bld = g.event_ms(lambda: L.sf_grav_tree_free(L.sf_grav_build_tree(dx, dm, dh, o)), 5)
            t = L.sf_grav_build_tree(dx, dm, dh, o)
            fwd = g.event_ms(lambda: L.sf_grav_accel(t, None, None, None, o), 10)
            bwd = g.event_ms(lambda: L.sf_grav_accel_backward(t, None, None, None, o, dga, dgp), 5)
            L.sf_grav_tree_free(t)
            others["diff256k"][form] = {"build_ms": bld, "accel_ms": fwd, "backward_ms": bwd,
                                        "backward_over_accel": bwd / fwd,
                                        "with_build": (bwd + bld) / (fwd + bld)}
            log(f"diff256k adjoint {form}: build {bld:.2f} ms, accel {fwd:.2f} ms, backward "
                f"{bwd:.2f} ms, ratio {bwd / fwd:.2f}")
        del dx, dm, dh, dga, dgp
        torch.cuda.empty_cache()
        if not args.no_fractal:
            others["fractal16m"] = fractal_leg(g, caps, alpha, keep)

    # oracle results
    cpu, errs = None, {}
    if worker is not None:
        rc = worker.wait(timeout=900)
        if rc != 0:
            log(f"oracle worker failed with status {rc}")
        for name in names:
            try:
                ref = np.load(os.path.join(outdir, f"{name}_ref.npy"))
                smp = np.load(os.path.join(outdir, f"{name}_sample.npy"))
                meta = json.load(open(os.path.join(outdir, f"{name}.json")))
            except OSError:
                continue
            assert np.array_equal(smp, samples[name])
            for (wname, leg), got in kept.items():
                if wname == name:
                    errs.setdefault(name, {})[leg] = errors(np, got, ref)
                    e = errs[name][leg]
                    log(f"error {name} {leg}: median {e['median']:.3e}, p99 {e['p99']:.3e}")
            if name == "precision4m":
                for leg, fname in (("T", "precision4m_tidal_T.npy"), ("j", "precision4m_tidal_J.npy")):
                    try:
                        ref_t = np.load(os.path.join(outdir, fname))
                    except OSError:
                        continue
                    got = kept.get(("precision4m_tidal", leg))
                    if got is not None:
                        tidal["rel_err_" + leg] = errors(np, got, ref_t)
                        log(f"error precision4m tidal {leg}: median "
                            f"{tidal['rel_err_' + leg]['median']:.3e}, p99 "
                            f"{tidal['rel_err_' + leg]['p99']:.3e}")
                cpu = {"value": meta["targets"] / meta["seconds"], "unit": "accels/s",
                       "cores": meta["threads"], "kind": "oracle",
                       "cpu": cpu_model(),
                       "sample": f"first {meta['targets']} of the {smp.size} random targets "
                                 f"x all {meta['sources']} sources, FP64 direct sum, "
                                 f"{meta['seconds']:.1f}s on {meta['threads']} threads "
                                 f"(run beside the GPU legs)"}

    achieved = walk_flop / (walk32 * 1e-3) / 1e12
    pmc = stored_walk_traffic()
    traffic = pmc["bytes_per_launch"] if pmc else None
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
                   "path": "tree", "theta": args.theta, "alpha": alpha, "order": "quadrupole",
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
        # second-stream intervals, fork to join, waiting included (not kernel
        # cost; the standalone sink work is tree_pass_extras.sinks_pass_ms)
        "side_stream_span_ms": side32,
        # per timed step (each synchronised): median and minimum beside the mean
        "step_stats": step_stats,
        # the whole step against its ideal time at peak: algorithmic walk FLOP
        # at the FP32 peak, build and walk bytes at the HBM peak (the larger)
        "step_roofline_frac": max(walk_flop / (PEAK_FP32_TFLOPS * 1e12),
                                  (SORT_BYTES_PER_PARTICLE + WALK_BYTES_PER_PARTICLE) * ps.n
                                  / (PEAK_HBM_GBS * 1e9)) / wall32,
    }
    if clocks:
        line["gfx_clock_mhz"] = clocks
    sort_ms = ph32.get("sort")
    if sort_ms:
        gbs = SORT_BYTES_PER_PARTICLE * ps.n / (sort_ms * 1e-3) / 1e9
        line["build_sort_hbm"] = {"bytes_per_particle": SORT_BYTES_PER_PARTICLE,
                                  "achieved_gbs": gbs, "frac": gbs / PEAK_HBM_GBS}
    for key, v in res.items():
        line[key] = v
    if "fp64" in res:
        line["fp32c_over_fp64"] = res["fp64"]["ms_per_step"] / (wall32 * 1e3)
    if adj:
        line["adjoint"] = adj
    if direct:
        line["direct"] = direct
    if tidal:
        line["tidal_jerk"] = tidal
    if extra:
        line["tree_pass_extras"] = extra
    line.update(others)
    if errs:
        line["rel_err"] = errs
        e = errs.get("precision4m", {}).get("tree_fp32c")
        if e:
            line["rel_err_fp32c"] = e
            line["p99_bar_1e-3_met"] = e["p99"] <= 1e-3
    print(json.dumps(line), flush=True)


def make_workload_size(name):
    return {"uniform4k": 4096, "clustered1m": (1 << 20) + 256, "precision4m": (1 << 22) + 4096,
            "fractal16m": (1 << 24) + 10000}[name]


def direct_leg(g, ps, x, m, h, head, keep, clocks):
    """Direct path at the workload's full size: one evaluation per form over
    all pairs, timed with HIP events, outputs kept for the error check."""
    L, torch = g.L, g.torch
    direct = {}
    pairs = ps.n_gas * ps.n + ps.n_sink * ps.n_gas
    acc, pot = head.acc[0], head.pot
    for form in ("fp32c", "fp32", "fp64"):
        o = L.make_opts(form=form, n_gas=ps.n_gas)
        k = 65536
        L.sf_grav_accel(None, x[:k].contiguous(), m[:k].contiguous(), h[:k].contiguous(),
                        L.make_opts(form=form, n_gas=k), acc=acc[:k], pot=pot[:k])  # warm
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        with ClockSampler() as cs:   # the graphics clock during the evaluation
            a.record()
            L.sf_grav_accel(None, x, m, h, o, acc=acc, pot=pot)
            b.record()
            torch.cuda.synchronize()
        if form == "fp32c":
            clocks["direct_fp32c"] = cs.summary()
        ms = a.elapsed_time(b)
        keep("precision4m", "direct_" + form, acc)
        tf = FLOP_PP * pairs / (ms * 1e-3) / 1e12
        peak = PEAK_FP64_TFLOPS if form == "fp64" else PEAK_FP32_TFLOPS
        direct[form] = {"ms": ms, "value": ps.n / (ms * 1e-3), "pairs_per_s": pairs / (ms * 1e-3),
                        "achieved_tflops": tf, "peak": peak, "frac": tf / peak}
        if form != "fp64":
            direct[form]["frac_nonpacked"] = tf / PEAK_FP32_NONPACKED_TFLOPS
        log(f"direct {form}: {ms:.1f} ms, {pairs / (ms * 1e-3):.3e} pairs/s, {tf:.1f} TFLOP/s")
    direct["fp32c_over_fp64"] = direct["fp64"]["ms"] / direct["fp32c"]["ms"]
    return direct


def fractal_leg(g, caps, alpha, keep):
    """fractal16m (16,777,216 gas in a 3-level Plummer-in-Plummer hierarchy +
    10,000 sinks, seed 4): forward and backward at theta 0.5 and 0.7,
    FP32C against FP64 (theta only, as the workload specifies), and the
    FP32C step with the relative criterion at theta 0.5."""
    np, torch, L = g.np, g.torch, g.L
    from synth import cotangents
    t0 = time.time()
    ps = make_workload("fractal16m")
    log(f"fractal16m: {ps.n} particles generated in {time.time() - t0:.1f}s")
    x, m, h = g.upload(ps)
    ga, gp = (torch.as_tensor(v).to(g.dev) for v in cotangents(ps.n, seed=4, dtype=np.float32))
    out = {"n": ps.n, "n_gas": ps.n_gas, "n_sink": ps.n_sink, "seed": 4}
    for theta, al in ((0.5, None), (0.7, None), (0.5, alpha)):
        for form in ("fp32c", "fp64"):
            if al is not None and form == "fp64":
                continue
            leg = TreeLeg(g, ps, x, m, h, form, theta, al, **caps)
            wall, ph = leg.timed(3, 1)
            key = f"theta{theta}_{form}" + ("_relative" if al is not None else "")
            keep("fractal16m", key, leg.last)
            r = {"ms_per_step": wall * 1e3, "value": ps.n / wall, "walk_ms": ph.get("walk"),
                 "alpha": al}
            if form == "fp32c":
                st, _ = leg.stats()
                r["n_pc"], r["n_pp"] = st["n_pc"], st["n_pp"]
                r["walk_tflops"] = (FLOP_PP * st["n_pp"] + FLOP_PC[2] * st["n_pc"]) / (
                    ph["walk"] * 1e-3) / 1e12
            t, o = leg.handle()
            r["accel_ms"] = g.event_ms(lambda: L.sf_grav_accel(t, None, None, None, o,
                                                               acc=leg.acc[0], pot=leg.pot), 2)
            r["backward_ms"] = g.event_ms(lambda: L.sf_grav_accel_backward(t, None, None, None, o,
                                                                           ga, gp), 1)
            r["backward_over_accel"] = r["backward_ms"] / r["accel_ms"]
            L.sf_grav_tree_free(t)
            out[key] = r
            log(f"fractal16m {key}: step {wall * 1e3:.1f} ms, accel {r['accel_ms']:.1f} ms, "
                f"backward {r['backward_ms']:.1f} ms")
            del leg
        if al is None:
            out[f"theta{theta}_fp32c_over_fp64"] = (out[f"theta{theta}_fp64"]["ms_per_step"] /
                                                    out[f"theta{theta}_fp32c"]["ms_per_step"])
    del x, m, h, ga, gp
    torch.cuda.empty_cache()
    return out


if __name__ == "__main__":
    main()
