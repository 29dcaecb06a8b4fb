"""Benchmark of the world step on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu] [--no-variants]

Workload: the 1024x1024 torus started with 65,536 agents (capacity 131,072),
11x11x4 window + 8 scalars, per-agent 492->64->64->7 MLP, FP32 weights, with
the full dynamics (costs, eating, deaths, births with mutation, regrowth).
One step = one pass of the whole hot path (policy forward, sampling, moves,
eating, births/deaths, regrowth, compaction/statistics) over all live agents.

value = live agent-steps per second (sum over the timed steps of the agents
alive at each step's start, divided by the wall time of the timed region,
inputs resident in HBM); the timed region replays hipGraphs of whole steps
(K steps as 32-step graphs and one of the remainder), the library's default
path.  The roofline object reports the policy
kernel (the dominant kernel): algorithmic bytes (live agents x per-agent
weight and state bytes) over its average launch duration, measured with HIP
events on the library's stream over the next K steps, replayed from one graph
that carries event-record nodes around every policy-kernel launch (those nodes
slow the replay, so that region's own step time is reported apart as
timing_region_ms_per_step); it also gives the achieved rate as a fraction of
the box's streaming-read rate, measured by the library's probe kernel (8 GiB
read once per launch; best of three calls of five launches at three grid shapes).  Also reported: BF16 and FP8 weight storage on the
same world, the frozen-population form (exactly 65,536 agents every step), the
same world with attacks enabled (the paper's "+A" worlds, with its predation
measures: attacks per agent and homicides per attack), the same world with the
paper's own policy options (evolving softmax temperature, colour trait rendered
into the windows), the same grid and population in the three-resource ecology
with health, and with terrain and the paper's 7x7 colour window (with and
without full-strength attacks; the latter also with its population held at 65,536), a per-kernel
breakdown from a few eager steps,
and the CPU oracle on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, AMD published
STATE_BYTES_PER_AGENT = 24   # policy kernel's per-agent state traffic: live idx, pos, facing, energy, age, outputs


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_history(w, steps, s_end):
    """Agent-steps and population bookkeeping of the last `steps` steps (ending at s_end)."""
    out = dict(agent_steps=0, pop_start=0, pop_end=0, births=0, deaths=0, attacks=0, killed=0)
    for i in range(w.n_worlds):
        hist = w.stats_history(i, steps + 1)
        assert hist[-1]["step"] == s_end
        out["agent_steps"] += sum(h["population"] for h in hist[:-1])  # live at the start of each step
        out["pop_start"] += hist[0]["population"]
        out["pop_end"] += hist[-1]["population"]
        out["births"] += sum(h["births"] for h in hist[1:])
        out["deaths"] += sum(h["deaths"] for h in hist[1:])
        atk = 8 if w.A == 9 else 6   # the attack action: ninth in the ecology, seventh otherwise
        out["attacks"] += sum(h["action_hist"][atk] for h in hist[1:])
        out["killed"] += sum(h["killed"] for h in hist[1:])
    return out


TUNE_CACHE = os.path.join(ROOT, "paper_2510_18221_amd", "launch_cache.jsonl")


def timed_run(eco, cfg, steps, warmup, autotune=True, launch=None, tune_cache=None):
    import torch
    w = eco.World(cfg)
    if launch:
        w.set_launch(*launch)
    tuned = w.autotune(cache=tune_cache) if autotune else w.get_launch()
    # timed region: K steps replayed from hipGraphs of whole steps (the library's default path)
    w.set_flags(eco.RT_USE_GRAPH)
    w.prepare(steps)
    if warmup:
        w.step(warmup)
    torch.cuda.synchronize()
    s0 = w.stats()[0]["step"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    w.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    res = dict(seconds=t1 - t0, steps=steps, launch=tuned, info=w.info, **run_history(w, steps, s0 + steps))
    # kernel-timing region: the next K steps from one hipGraph that carries HIP
    # event-record nodes around every policy-kernel launch (on the library's
    # stream).  Those nodes cost the replay tens of microseconds per step, which
    # is why the throughput above comes from the graph without them.
    w.set_flags(eco.RT_USE_GRAPH | eco.RT_TIME_KERNELS)
    w.prepare(steps)
    w.kernel_times(reset=True)
    s1 = w.stats()[0]["step"]
    torch.cuda.synchronize()
    u0 = time.perf_counter()
    w.step(steps)
    torch.cuda.synchronize()
    u1 = time.perf_counter()
    res["kernel_times"] = w.kernel_times(reset=True)
    res["timing_region"] = dict(seconds=u1 - u0, **run_history(w, steps, s1 + steps))
    # per-kernel breakdown: a few eager steps with events around every kernel group
    w.set_flags(eco.RT_TIME_KERNELS)
    n_eager = min(steps, 10)
    s2 = w.stats()[0]["step"]
    w.step(n_eager)
    res["kernel_times_eager"] = w.kernel_times(reset=True)
    res["eager"] = run_history(w, n_eager, s2 + n_eager)
    res["eager"]["steps"] = n_eager
    # births of every step of the run, oldest first (the birth kernel's launches, one per step)
    res["births_per_step"] = [h["births"] for h in w.stats_history(0, 1024)[1:]] if w.n_worlds == 1 else None
    w.close()
    torch.cuda.empty_cache()
    return res


def trajectory(eco, cfg, steps, chunk=1000, out_path=None, tune_cache=None):
    """Long free-running run: population, throughput and policy-kernel bandwidth per chunk
    of steps (each chunk replayed from one graph with event nodes around the policy kernel).
    The launch shape is chosen again before each chunk for the live population of the
    moment (the tuner's cache is keyed by its power-of-two bucket)."""
    import torch
    w = eco.World(cfg)
    w.set_flags(eco.RT_USE_GRAPH | eco.RT_TIME_KERNELS)
    bytes_per_agent = w.info["weight_bytes_per_agent"] + STATE_BYTES_PER_AGENT
    rows = []
    for c0 in range(0, steps, chunk):
        n = min(chunk, steps - c0)
        launch = w.autotune(cache=tune_cache)
        w.set_flags(eco.RT_USE_GRAPH | eco.RT_TIME_KERNELS)
        w.prepare(n)
        w.kernel_times(reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        w.step(n)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        fwd_ms = w.kernel_times(reset=True)["forward"][0]
        hist = w.stats_history(0, n + 1)
        agent_steps = sum(h["population"] for h in hist[:-1])
        row = {"step": hist[-1]["step"], "population": hist[-1]["population"],
               "births": sum(h["births"] for h in hist[1:]), "deaths": sum(h["deaths"] for h in hist[1:]),
               "agent_steps_per_s": round(agent_steps / dt, 1), "ms_per_step": round(dt * 1e3 / n, 4),
               "forward_GBps": round(agent_steps * bytes_per_agent / (fwd_ms * 1e-3) / 1e9, 1) if fwd_ms > 0 else 0.0,
               "pop_min": min(h["population"] for h in hist), "pop_max": max(h["population"] for h in hist),
               "launch": [launch["waves_per_block"], launch["blocks_per_cu"], launch["unroll"]]}
        rows.append(row)
        log(f"[trajectory] {row}")
    w.close()
    torch.cuda.empty_cache()
    if out_path:
        with open(out_path, "w") as f:
            json.dump(rows, f, indent=1)
    return rows


def profiled_traffic(name):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or None
    when the policy kernel's source changed since the counters were taken."""
    from paper_2510_18221_amd import rocprof_summary
    path = os.path.join(ROOT, "profiles", f"k_forward_{name}_hbm_traffic.md")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and line.split(":")[0] in ("traffic_bytes_per_launch", "source_sha256"):
            k, v = line.split(":", 1)
            vals[k] = v.strip()
    if vals.get("source_sha256") != rocprof_summary.forward_source_sha():
        return None
    return float(vals["traffic_bytes_per_launch"])


READ_CEILING = {}  # measured once per run: the library's streaming-read probe
COPY_CEILING = {}  # measured once per run: a device-to-device copy (half reads, half writes)


def measure_copy_ceiling(nbytes=4 << 30, reps=5):
    """Read + write bytes per second of torch's device copy of nbytes (best of reps),
    the ceiling of a kernel whose traffic is half reads and half writes."""
    import torch
    x = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    best = float("inf")
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        y.copy_(x)
        b.record()
        b.synchronize()
        best = min(best, a.elapsed_time(b) * 1e-3)
    del x, y
    torch.cuda.empty_cache()
    return 2 * nbytes / best / 1e9


def roofline(r, profile_name=None):
    ms, n = r["kernel_times"]["forward"]
    avg_ms = ms / max(n, 1)
    agents_per_launch = r["timing_region"]["agent_steps"] / max(n, 1)
    bytes_per_agent = r["info"]["weight_bytes_per_agent"] + STATE_BYTES_PER_AGENT
    gbs = agents_per_launch * bytes_per_agent / (avg_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4),
            "traffic": profiled_traffic(profile_name) if profile_name else None,
            "kernel": "k_forward", "avg_launch_ms": round(avg_ms, 4),
            "bytes_per_agent": bytes_per_agent, "agents_per_launch": round(agents_per_launch, 1),
            "measured_read_ceiling_GBps": READ_CEILING.get("gbps"),
            "frac_of_measured_ceiling": round(gbs / READ_CEILING["gbps"], 4) if READ_CEILING.get("gbps") else None}


def birth_roofline(r):
    """The birth-commit kernel over the eager steps (HIP events around each launch):
    algorithmic bytes per birth = the parent's FP32 master read (4P), the child's
    master written (4P) and, when the storage is a separate BF16 / FP8 copy, that
    copy written (the per-agent weight bytes of the forward)."""
    ms, n = r["kernel_times_eager"]["birth_commit"]
    births = r["eager"]["births"]
    info = r["info"]
    P = info["param_count"]
    per_birth = 8 * P + (info["weight_bytes_per_agent"] if info["wdtype"] != 0 else 0)
    avg_ms = ms / max(n, 1)
    per_launch = births / max(n, 1)
    gbs = per_launch * per_birth / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    out = {"bound": "hbm", "kernel": "k_birth_commit", "births_per_launch": round(per_launch, 1),
           "bytes_per_birth": per_birth, "avg_launch_ms": round(avg_ms, 4), "achieved": round(gbs, 1),
           "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4)}
    if COPY_CEILING.get("gbps"):
        out["measured_copy_ceiling_GBps"] = COPY_CEILING["gbps"]
        out["frac_of_measured_copy_ceiling"] = round(gbs / COPY_CEILING["gbps"], 4)
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(min_seconds=10.0, max_steps=100):
    """The oracle as it stands, on a bounded sample of the same workload: the
    same 65,536-agent world (init not timed), stepped until ~10 s of CPU work
    with OpenMP over agents on all threads, then ~10 s more on one thread."""
    import ctypes
    from oracle import oracle as orc
    from paper_2510_18221_amd import workloads as wl
    cfg = wl.world_65k(seed=0)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    w = orc.OracleWorld(cfg)

    def sample(seconds):
        pops = []
        t0 = time.perf_counter()
        while len(pops) < max_steps and (time.perf_counter() - t0 < seconds or len(pops) < 2):
            pops.append(w.stats()["population"])
            w.step()
        return pops, time.perf_counter() - t0

    pops, dt = sample(min_seconds)
    gomp = ctypes.CDLL("libgomp.so.1")  # the OpenMP runtime the oracle library runs on
    gomp.omp_set_num_threads(1)
    pops1, dt1 = sample(min_seconds)
    gomp.omp_set_num_threads(threads)
    w.close()
    return {"value": round(sum(pops) / dt, 1), "unit": "agent-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"the same 1024x1024 world with 65,536 agents, FP32 weights, {len(pops)} full steps "
                      f"(policy sampled by the oracle) after an untimed init; FP64 policy with OpenMP over "
                      f"agents, sequential world update",
            "seconds": round(dt, 2),
            "single_thread": {"value": round(sum(pops1) / dt1, 1), "steps": len(pops1), "seconds": round(dt1, 2)},
            "host": {"cpu_model": cpu_model(), "logical_cpus": os.cpu_count(),
                     "usable_cpus": len(os.sched_getaffinity(0))}}


WORKLOADS = {
    "65k": ("single world 1024x1024 torus, 65,536 agents at start, capacity 131,072, 11x11x4 window + 8 "
            "scalars, per-agent 492->64->64->7 MLP, FP32 weights; every kernel of the step runs, but with energy "
            "starting at 10, a cost of 0.1 per step and reproduction at 20 no agent is born or dies in the "
            "timed steps (births and deaths are timed in the turnover and ecology variants)", "f32"),
    "batch": ("64 independent worlds in one object (one graph per step), sides log-uniform in [128, 1024], 6.25% "
              "occupancy (984,579 agents), capacity 1.125x, 492->64->64->7 BF16 weights + FP32 master", "bf16"),
    "large": ("single world 2048x2048, capacity 262,144 starting half full, density 0.03, regrowth 0.005, "
              "15x15x4 window + 8 scalars, 908->128->128->7 BF16 weights + FP32 master", "bf16"),
    "small": ("single world 64x64 torus, 256 agents at start, capacity 4,096, density 0.1, regrowth 0.01, "
              "5x5x4 window + 4 scalars, 104->32->32->5 FP32 weights (cache-resident: a latency test)", "f32"),
    "small_ecology": ("single world 64x64 torus with the three-resource ecology, terrain (water flowing downhill) "
                      "and the 7x7 rendered colour + elevation window, 256 agents held (no costs, no births, no "
                      "health damage), 208->32->32->8 FP32 weights (cache-resident: a latency test)", "f32"),
    "turnover": ("single world 1024x1024 torus, 65,536 agents at start, capacity 131,072, 11x11x4 window + 8 "
                 "scalars, per-agent 492->64->64->7 MLP, FP32 weights; no step cost and no transfer to the "
                 "child (every agent at the reproduction threshold, children born with zero energy die at "
                 "their first step): a steady stream of ~9k births with mutation and as many deaths per step",
                 "f32"),
}
# the turnover world's changes to the 65k world's energies
TURNOVER = dict(e_init=200, e_cost=0, e_child=0)


def workload_cfg(wl, name, wdtype=None):
    wdt = {None: wl.FP32, "f32": wl.FP32, "bf16": wl.BF16, "fp8": wl.FP8}[wdtype]
    if name == "65k":
        return wl.world_65k(seed=0, wdtype=wdt)
    if name == "turnover":
        return dict(wl.world_65k(seed=0, wdtype=wdt), **TURNOVER)
    if name == "batch":
        return wl.world_batch(64)
    if name == "small":
        return wl.world_small(seed=0)
    if name == "small_ecology":
        held = dict(wl.ECOLOGY, e_cost_move=0, w_cost=0, hp_overspend=0, age_shift=31, attack_damage=0)
        return wl.ecology_desc(eco=held, window=7, n_scalars=12, e_cost=0, e_repro=1 << 30, seed=0,
                               flags=wl.ECOLOGY_FLAG | 16 | 4)   # with terrain and colour vision
    return wl.world_large(seed=0)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="65k")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--retune", action="store_true",
                    help="time the launch shapes instead of taking them from the tuner's result cache")
    ap.add_argument("--tune-cache", default=TUNE_CACHE, help="the tuner's result cache (JSON lines)")
    ap.add_argument("--wdtype", choices=["f32", "bf16", "fp8"], default=None,
                    help="weight storage of the 65k world's main line (default FP32, the metric's form)")
    ap.add_argument("--copy-probe", action="store_true", help="also run a plain 4 GiB device copy (PMC scaling)")
    ap.add_argument("--agents", type=int, default=0,
                    help="the 65k world's grid with this many agents instead, held (no cost, no births)")
    ap.add_argument("--launch", default=None, help="fixed policy-kernel launch 'waves_per_block,blocks_per_cu,unroll'")
    ap.add_argument("--trajectory", type=int, default=0, help="instead: free-run this many steps, report per 1000")
    ap.add_argument("--trajectory-out", default=None)
    ap.add_argument("--trajectory-chunk", type=int, default=1000, help="steps per trajectory row")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: worlds shard across GPUs by design but no multi-GPU path is "
              "built; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2510_18221_amd import eco
    from paper_2510_18221_amd import workloads as wl
    assert torch.cuda.is_available(), "bench needs a GPU"
    eco.lib()
    READ_CEILING["gbps"] = round(max(eco.stream_read_gbps(8 << 30) for _ in range(3)), 1)
    log(f"[bench] streaming-read ceiling {READ_CEILING['gbps']} GB/s")
    if args.workload in ("65k", "turnover"):
        COPY_CEILING["gbps"] = round(measure_copy_ceiling(), 1)
        log(f"[bench] device-copy ceiling {COPY_CEILING['gbps']} GB/s (reads + writes)")

    cfg = workload_cfg(wl, args.workload, args.wdtype)
    if args.agents:
        cfg = dict(wl.world_65k(seed=0, frozen=True, wdtype=cfg["wdtype"]), n_agents_init=args.agents)
    if args.trajectory:
        rows = trajectory(eco, cfg, args.trajectory, chunk=args.trajectory_chunk, out_path=args.trajectory_out,
                          tune_cache=None if args.retune else args.tune_cache)
        print(json.dumps({"workload": args.workload, "trajectory": rows}), flush=True)
        return

    log(f"[bench] {args.workload}: warmup {args.warmup}, timed {args.steps}")
    launch = tuple(int(v) for v in args.launch.split(",")) if args.launch else None
    autotune = not args.no_autotune and launch is None
    cache = None if args.retune else args.tune_cache
    main_r = timed_run(eco, cfg, args.steps, args.warmup, autotune=autotune, launch=launch, tune_cache=cache)
    value = main_r["agent_steps"] / main_r["seconds"]
    ms_per_step = main_r["seconds"] * 1e3 / main_r["steps"]
    log(f"[bench] {args.workload}: {value / 1e6:.2f} M agent-steps/s, {ms_per_step:.3f} ms/step, "
        f"launch {main_r['launch']}")
    desc, dtype = WORKLOADS[args.workload]
    if args.workload in ("65k", "turnover") and args.wdtype in ("bf16", "fp8"):
        desc = desc.replace("FP32 weights", {"bf16": "BF16 weights + FP32 master",
                                             "fp8": "FP8-E4M3 weights + row scales + FP32 master"}[args.wdtype])
        dtype = args.wdtype
    out = {
        "metric": "agent-steps/s at 65,536 agents, FP32 vs BF16 weights; % of HBM peak",
        "value": round(value, 1), "unit": "agent-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic",
        "config": {"workload": desc, "agents_start": main_r["pop_start"], "agents_end": main_r["pop_end"],
                   "births": main_r["births"], "deaths": main_r["deaths"], "launch": main_r["launch"]},
        "roofline": roofline(main_r, {None: "65k_fp32", "f32": "65k_fp32", "bf16": "65k_bf16",
                                      "fp8": "65k_fp8"}[args.wdtype] if args.workload == "65k" else None),
        "world_steps_per_s": round(1e3 / ms_per_step, 1),
        "timing_region_ms_per_step": round(main_r["timing_region"]["seconds"] * 1e3 / main_r["steps"], 4),
        "kernel_ms_per_step_eager": {k: round(v[0] / max(v[1], 1), 4)
                                     for k, v in main_r["kernel_times_eager"].items()},
    }
    if args.workload == "turnover":
        out["config"]["births_deaths"] = [main_r["births"], main_r["deaths"]]
        out["birth_roofline"] = birth_roofline(main_r)
        out["births_per_step"] = main_r["births_per_step"]
    if args.workload == "65k" and not args.no_variants:
        variants = {}
        attack_cfg = dict(wl.world_65k(seed=0), attack_enabled=1)
        # the paper's own agent: evolving softmax temperature and colour trait seen in others' windows
        paper_cfg = dict(wl.world_65k(seed=0), flags=eco.DESC_EVOLVE_TEMPERATURE | eco.DESC_COLOUR_VISION)
        # the three-resource ecology with health on the same grid and population (496->64->64->8)
        ecology_cfg = wl.ecology_desc(width=1024, height=1024, n_agents_init=65536, capacity=131072, window=11,
                                      n_scalars=12, hidden1=64, hidden2=64, mutation_sigma=0.01, e_init=230, seed=0)
        # the paper's vision agent (RCV) in a world with terrain: a 7x7 window of rendered colour and
        # elevation difference, the compass, the ecology with water flowing downhill (208->64->64->8)
        terrain_cfg = dict(ecology_cfg, window=7, flags=eco.DESC_ECOLOGY | eco.DESC_TERRAIN | eco.DESC_COLOUR_VISION)
        # the paper's "Ocean" agent (RCV+A): the same, with full-strength attacks as a ninth action and the
        # paper's evolving softmax temperature (208->64->64->9, + log tau)
        ocean_cfg = dict(terrain_cfg, n_actions=9, attack_enabled=1,
                         flags=terrain_cfg["flags"] | eco.DESC_EVOLVE_TEMPERATURE)
        # the same agent with the population held at 65,536 (no costs, no births, harmless strikes: the same
        # kernels, their cost at full size)
        ocean_held_cfg = dict(ocean_cfg, e_cost=0, e_repro=1 << 30,
                              eco=dict(ocean_cfg["eco"], e_cost_move=0, w_cost=0, hp_overspend=0, age_shift=31,
                                       attack_damage=0))
        # a steady birth stream at ~65k agents: no step cost and no transfer, so every agent stays at
        # the reproduction threshold and a parent needs only the REPRODUCE action and a free cell behind
        # it; children start with zero energy and die at their first step, so ~9k births with mutation
        # into recycled slots and as many deaths happen every step
        turnover = TURNOVER
        for name, vcfg in [("bf16", wl.world_65k(seed=0, wdtype=wl.BF16)),
                           ("fp32_turnover", dict(wl.world_65k(seed=0), **turnover)),
                           ("bf16_turnover", dict(wl.world_65k(seed=0, wdtype=wl.BF16), **turnover)),
                           ("fp8", wl.world_65k(seed=0, wdtype=wl.FP8)),
                           ("fp32_frozen", wl.world_65k(seed=0, frozen=True)),
                           ("fp32_attack", attack_cfg),
                           ("fp32_temperature_colour", paper_cfg),
                           ("fp32_ecology", ecology_cfg),
                           ("fp32_terrain_rcv_7x7", terrain_cfg),
                           ("fp32_terrain_rcv_a_7x7", ocean_cfg),
                           ("fp32_terrain_rcv_a_7x7_held", ocean_held_cfg)]:
            log(f"[bench] variant {name}")
            r = timed_run(eco, vcfg, args.steps, args.warmup, autotune=autotune, launch=launch, tune_cache=cache)
            v = r["agent_steps"] / r["seconds"]
            variants[name] = {"value": round(v, 1), "ms_per_step": round(r["seconds"] * 1e3 / r["steps"], 4),
                              "roofline": roofline(r, {"bf16": "65k_bf16", "fp8": "65k_fp8"}.get(name)),
                              "agents_start": r["pop_start"], "agents_end": r["pop_end"],
                              "launch": r["launch"]}
            if vcfg.get("flags", 0) & eco.DESC_ECOLOGY or name.endswith("turnover"):
                variants[name]["births_deaths"] = [r["births"], r["deaths"]]
                if r["eager"]["births"]:   # the birth kernel's rate, over the eager steps' births
                    variants[name]["birth_roofline"] = birth_roofline(r)
            if vcfg.get("attack_enabled"):
                # the predation measures of the paper's Table 3 over the timed steps
                variants[name]["attacks_per_agent"] = round(r["attacks"] / max(r["agent_steps"], 1), 4)
                variants[name]["homicides_per_attack"] = round(r["killed"] / max(r["attacks"], 1), 4)
            log(f"[bench] {name}: {v / 1e6:.2f} M agent-steps/s")
        # the batching pattern (64 independent worlds of uneven size, one graph per step) and the large world
        for name, wname in [("batch64_bf16", "batch"), ("large2048_bf16", "large")]:
            log(f"[bench] variant {name}")
            r = timed_run(eco, workload_cfg(wl, wname), args.steps, args.warmup, autotune=autotune, launch=launch,
                          tune_cache=cache)
            v = r["agent_steps"] / r["seconds"]
            variants[name] = {"value": round(v, 1), "ms_per_step": round(r["seconds"] * 1e3 / r["steps"], 4),
                              "workload": WORKLOADS[wname][0],
                              "roofline": roofline(r), "agents_start": r["pop_start"], "agents_end": r["pop_end"],
                              "births_deaths": [r["births"], r["deaths"]], "launch": r["launch"]}
            log(f"[bench] {name}: {v / 1e6:.2f} M agent-steps/s")
        out["variants"] = variants
    if args.copy_probe:
        x = torch.empty(1 << 30, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    if args.workload == "65k" and not args.no_cpu:
        log("[bench] CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
