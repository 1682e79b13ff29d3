"""Benchmark of one ADG time step (three SSP-RK3 stages, every hot-path step) on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c1|c0|c2]

A "step" is one full SSP-RK3 time step: three fused stage launches (DG right-hand
side, chemistry, AT fluxes at PE interfaces, RK update, history publish; for the
limited workload also the KXRCF/AT-WENO limiter of the stage's output).  The
metric counts scalar DOF updates (E (N_p+1) (3+N_s) per stage) per second, with
the inputs resident in HBM before the timed region starts.

Prints ONE JSON line.  The roofline object refers to the dominant kernel (the
stage kernel): its average launch duration is measured with HIP events that the
library records on the solver's stream around every launch (adg_profile).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DOF-updates/s per RK stage (plain vs batched mixed); p50/p99 solve latency"
RK_STAGES = {"ssprk3": 3, "rk2": 2, "lserk4": 5}
HBM_PEAK_GBS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6


def workload(name: str, n_elem: int | None = None):
    from workloads import gen

    kw = {} if n_elem is None else {"E": n_elem}
    if name == "c0":
        case, w0 = gen.case_c0(**kw)
    elif name == "c1":
        case, w0 = gen.case_c1(**kw)
    elif name == "c2":
        case, w0 = gen.case_c2(**kw)
    else:
        raise SystemExit(f"unknown workload {name}")
    return case, w0


COPY_PROBE_BYTES = 256 * 1024 * 1024


def pmc_probe(args):
    """Run under rocprofv3 --pmc: one plain device copy of COPY_PROBE_BYTES (the calibration
    kernel for FETCH_SIZE / WRITE_SIZE), two launches of the FP64 FMA-chain kernel
    (peaks.adg_peak_fp64_fmas() FMAs each: the calibration of the FP64 instruction
    counters), then args.steps time steps with plain launches."""
    import torch

    from paper_2501_01747_amd import adg, peaks

    src = torch.ones(COPY_PROBE_BYTES // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    peaks.fp64_rate(n_reps=1)
    torch.cuda.synchronize()
    if args.workload == "c3":
        b, cases = build_c3_batch(args.precision)
        b.step(args.steps)
        b.poll()
        b.close()
        print(json.dumps({"probe": "c3_batched_ignition", "instances": len(cases), "copy_bytes": COPY_PROBE_BYTES,
                          "steps": args.steps}), flush=True)
        return
    case, w0 = workload(args.workload, args.n_elem)
    s = adg.Solver(case)
    s.set_state(w0)
    s.step(args.steps)
    s.sync()
    print(json.dumps({"probe": case["name"], "n_elem": case["disc"]["n_elem"], "copy_bytes": COPY_PROBE_BYTES,
                      "steps": args.steps}), flush=True)


def euler_stage_bytes(case) -> float:
    """Algorithmic HBM bytes of one stage launch, averaged over the three stages:
    stage 1 reads w^n and writes w^(1) (16 B/DOF); stages 2 and 3 read w^n and
    w^(s) and write w^(s+1) (24 B/DOF); with the limiter (inside the same kernel)
    one troubled-cell flag byte per element."""
    from workloads import gen

    flags = case["disc"]["n_elem"] if case["disc"].get("limiter") else 0
    return gen.dof(case) * 8.0 * (2 + 3 + 3) / 3.0 + flags


def detailed_stage_flops(case) -> float:
    """Algorithmic FP64 operations of one detailed-chemistry stage launch (count of
    +, -, *, / and one per exp/log/pow), from the formulas evaluated per element:

      per quadrature node (Q = N_p+1 per element) and per face trace (2 per element):
        temperature Newton, 4 iterations x Ns x (cp, h polynomials: 20)       = 80 Ns
        primitives, pressure, sound speed                                      = 10 + 4 Ns
        diffusive flux (gradients, transport law, heat flux)                   = 30 + 8 Ns
        convective flux                                                        = 4 + Ns
      per quadrature node only (chemistry):
        Gibbs energies 14 Ns, rates 21 reactions x (2 exp + 12)                = 14 Ns + 14 Nr
        species production 2 Nr Ns
      per element: modal->nodal interpolation 2 M (Q+2) V, LDG gradient 4 M M V,
        nodal->modal projection 2 M Q (V + Ns), lift + RK 8 M V
      per face: Rusanov 6 V + 8, central diffusive average 2 V
    """
    d = case["disc"]
    E, M = d["n_elem"], d["order_p"] + 1
    Q = M
    ns = case["physics"]["n_species"]
    nr = case["physics"]["mech"]["n_reactions"]
    V = 3 + ns
    point = 80 * ns + (10 + 4 * ns) + (30 + 8 * ns) + (4 + ns)
    chem = 14 * ns + 14 * nr + 2 * nr * ns
    elem = 2 * M * (Q + 2) * V + 4 * M * M * V + 2 * M * Q * (V + ns) + 8 * M * V
    face = 6 * V + 8 + 2 * V
    return float(E * ((Q + 2) * point + Q * chem + elem + face))


def src_hash(files) -> str:
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, "paper_2501_01747_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def read_traffic(name: str, kernel_src: list[str]):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3 --pmc summary
    (2 x FETCH_SIZE + WRITE_SIZE: FETCH_SIZE reads half of a plain copy's read bytes on this
    part), or None when missing or taken on a different version of the kernel source."""
    path = os.path.join(ROOT, "profiles", f"traffic_{name}.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"bytes_per_launch:\s*([0-9.eE+]+)", txt)
    h = re.search(r"kernel_src_sha:\s*([0-9a-f]+)", txt)
    if not m or not h or h.group(1) != src_hash(kernel_src):
        return None
    return float(m.group(1))


def cpu_baseline(case, w0, budget_s: float = 12.0):
    """The oracle as it stands, single thread, on the same workload from the same
    initial state: as many whole time steps as fit in about `budget_s`."""
    from oracle import oracle
    from workloads import gen

    oracle.build(force=not os.path.exists(oracle._LIB_PATH))
    cap = 100000
    s = oracle.OracleSolver(case, w0, cap)
    t0 = time.perf_counter()
    steps = 0
    chunk = 1
    while True:
        s.step(chunk)
        steps += chunk
        el = time.perf_counter() - t0
        if el >= budget_s or steps + chunk * 2 > cap:
            break
        if el < budget_s / 8:
            chunk *= 2
    s.close()
    rate = gen.dof(case) * 3 * steps / el
    return {"value": rate, "unit": "DOF-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} time steps of the same workload from the same initial state "
                      f"({el:.1f} s, single thread, gcc -O2)"}


def cpu_baseline_batch(cases, budget_s: float = 10.0, steps: int = 8):
    """The oracle as it stands on the batched workload's instances, one instance per host
    thread at a time (the oracle is a C library called through ctypes, which releases the
    interpreter lock): instances taken in order, `steps` time steps each, until about
    `budget_s` has passed.  Threads = the host cores this process may use, at most 16."""
    import threading

    from oracle import oracle
    from workloads import gen

    oracle.build(force=not os.path.exists(oracle._LIB_PATH))
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    lock = threading.Lock()
    state = {"next": 0, "work": 0.0, "done": 0}
    t0 = time.perf_counter()

    def worker():
        while True:
            with lock:
                if time.perf_counter() - t0 >= budget_s or state["next"] >= len(cases):
                    return
                c, w = cases[state["next"]]
                state["next"] += 1
            s = oracle.OracleSolver(c, w, steps + 1)
            s.step(steps)
            s.close()
            with lock:
                state["work"] += gen.dof(c) * 3 * steps
                state["done"] += 1

    pool = [threading.Thread(target=worker) for _ in range(threads)]
    for t in pool:
        t.start()
    for t in pool:
        t.join()
    el = time.perf_counter() - t0
    return {"value": state["work"] / el, "unit": "DOF-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{state['done']} of the batch's instances, {steps} time steps each, FP64, "
                      f"{threads} host threads ({el:.1f} s)"}


def build_c3_batch(precision: str, n_inst: int = 4096):
    from paper_2501_01747_amd import adg
    from workloads import gen

    cases = list(gen.case_c3(n_inst=n_inst, mech=gen.c1_mechanism()))
    heap = sum(adg.Batch.instance_bytes(c) for c, _ in cases)
    elems = sum(c["disc"]["n_elem"] for c, _ in cases)
    b = adg.Batch(len(cases), elems, heap, precision=precision)
    for c, w in cases:
        b.add(c, w)
    return b, cases


def batch_decompositions(steps: int, precision: str):
    """Time every work decomposition of the batched kernel on the batched workload (the
    autotuner's candidates): HIP events over `steps` plain steps each, after one untimed step."""
    import torch

    b, cases = build_c3_batch(precision)
    out = {}
    for cfg in range(2):
        b.set_decomposition(cfg)
        b.step(1)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record(b.stream)
        b.step(steps)
        ev1.record(b.stream)
        torch.cuda.synchronize()
        out[cfg] = ev0.elapsed_time(ev1) / (3 * steps)
        print(json.dumps({"decomposition": cfg, "tile_elems": (8, 4)[cfg], "launch_ms": out[cfg]}), flush=True)
    b.close()
    return out


def bench_batched(steps: int, warmup: int, graph: int, precision: str = "mixed", n_inst: int = 4096,
                  cpu: bool = False):
    """The batched ignition workload: n_inst instances (element counts log-uniform in
    [128, 4096], N_p in {2, 3}, 4-32 PEs, SAA delays k <= 2) in one batch; every stage of
    every instance is one batched launch.  Returns the measurement as a dict."""
    import torch

    from workloads import gen

    b, cases = build_c3_batch(precision, n_inst)
    elems = sum(c["disc"]["n_elem"] for c, _ in cases)
    tuned = b.autotune()
    graph = min(graph, steps)   # the timed steps: steps // graph replays, steps mod graph plain steps
    if graph:
        b.set_graph(graph)
    b.step(max(warmup, 1))      # the first step after set_graph captures the graphs
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(b.stream)
    b.step(steps)
    ev1.record(b.stream)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    st, er = b.poll()
    dof = sum(gen.dof(c) for c, _ in cases)
    # every instance is a detailed-chemistry one: a step is three launches of the batched
    # kernel, timed with HIP events over the timed region on the batch's stream
    stage_ms = ev0.elapsed_time(ev1) / (3 * steps)
    flops = sum(detailed_stage_flops(c) for c, _ in cases)
    achieved = flops / (stage_ms * 1e-3) / 1e12
    b.close()
    out = {
        "value": dof * 3 * steps / el, "unit": "DOF-updates/s", "ms_per_step": el * 1e3 / steps,
        "steps": steps, "warmup": warmup, "precision": precision,
        "config": {"workload": "c3_batched_ignition", "instances": len(cases), "elements": elems, "dof": dof,
                   "order_p": [2, 3], "graph_steps": graph,
                   "timed_graph_replays": steps // graph if graph else 0, "tile_elems": (8, 4)[tuned]},
        "state_errors": int(er.sum()), "steps_done_min": int(st[st >= 0].min()),
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
                     "traffic": read_traffic("c3", ["adg_ns.hip", "adg_ns.hpp"]), "kernel": "ns_batch_kernel",
                     "launch_ms": stage_ms, "flops_per_launch": flops},
    }
    if cpu:
        out["cpu_baseline"] = cpu_baseline_batch(cases)
    return out


# Arrival rate of the served stream: 0.7 x the saturation throughput of the server
# (all requests queued at t = 0), measured once with --calibrate and then fixed.
C4_RATE = 16.0   # 0.7 x 22.94 requests/s measured with --calibrate --requests 300


def bench_serve(n_req: int, rate, heap_gib: float, slots: int, chunk: int, precision: str,
                group_streams: int | None = None, graph_steps: int = 0):
    """Served stream of n_req requests (half ignition, half reacting shock; E log-uniform in
    [256, 65536], N_p in {1..4}, 100-2000 steps) arriving as a Poisson process at `rate`
    requests/s (all at t = 0 when rate is None: the saturation measurement)."""
    import numpy as np
    import torch

    from paper_2501_01747_amd import adg
    from paper_2501_01747_amd.serve import Request, Server, summarize
    from workloads import gen

    t_gen = time.perf_counter()
    raw = list(gen.c4_requests(n_req, rate))
    reqs = [Request(r["rid"], r["case"], r["w0"], r["steps"], r["arrival"]) for r in raw]
    t_gen = time.perf_counter() - t_gen
    b = adg.Batch(slots, 1 << 27, int(heap_gib * 2**30), precision=precision)
    if group_streams:
        b.set_group_streams(group_streams)
    srv = Server(b, chunk=chunk, graph_steps=graph_steps)
    torch.cuda.synchronize()
    res = srv.run(reqs)
    b.close()
    out = summarize(res)
    fails = {}
    for q, r in zip(raw, res):
        if not r.ok:
            key = f"{q['kind']}_p{q['case']['disc']['order_p']}"
            fails[key] = fails.get(key, 0) + 1
    by_kind = {}
    for kind in ("ignition", "shock"):
        lat = [r.latency for q, r in zip(raw, res) if r.ok and q["kind"] == kind]
        if lat:
            by_kind[kind] = {"n": len(lat), "p50_latency_s": float(np.percentile(lat, 50)),
                             "p99_latency_s": float(np.percentile(lat, 99))}
    out.update({"failed_by_kind_order": fails, "latency_by_kind": by_kind, "rate_req_per_s": rate, "heap_gib": heap_gib, "slots": slots, "chunk": chunk,
                "precision": precision, "rounds": srv.rounds, "max_active": srv.max_active,
                "input_generation_s": t_gen, "loop_seconds": srv.time_in, "graph_steps": graph_steps,
                "group_streams": group_streams or 4})
    return out


def region_stage_ms(s, steps: int, graph: int = 10) -> float:
    """Mean stage-launch duration of a solver whose step is three stage launches: HIP events
    on its stream around `steps` steps replayed from `graph`-step HIP graphs, after one
    untimed replay."""
    import torch

    s.set_graph(graph)
    s.step(graph)
    s.sync()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(s.stream)
    s.step(steps)
    ev1.record(s.stream)
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / (3 * steps)


def hbm_points(steps: int = 20):
    """The one-step stage kernels at sizes where HBM bounds them (the C0 physics at E = 2^22 without
    the limiter, the C2 physics at E = 2^21 with it), each with its roofline against 8 TB/s: mean
    launch time from HIP events over graph-replayed steps on the solver's stream."""
    out = {}
    for key, res, kernel, tkey in (("c0_physics_E4194304", sweep_euler([2**22], steps)[0], "euler_stage_kernel",
                                    "c0_4194304"),
                                   ("c2_physics_E2097152", sweep_limiter([2**21], steps)[0], "euler_lim_kernel",
                                    "c2_2097152")):
        out[key] = {"n_elem": res["n_elem"], "dof": res["dof"], "launch_ms": res["stage_ms"],
                    "roofline": {"bound": "hbm", "kernel": kernel, "achieved": res["GBps"], "peak": HBM_PEAK_GBS,
                                 "unit": "GB/s", "frac": res["frac_hbm"], "bytes_per_launch": res["bytes"],
                                 "traffic": read_traffic(tkey, ["adg_euler.hip", "adg_device.hpp"])}}
    return out


def served_short(n_req: int, rate: float, precision: str):
    """A short served stream (n_req requests at the fixed arrival rate) for the default line."""
    out = bench_serve(n_req, rate, 16.0, 1024, 10, precision, graph_steps=2)
    keep = ("requests", "completed_ok", "failed", "p50_latency_s", "p99_latency_s", "mean_latency_s", "mean_queue_s",
            "makespan_s", "requests_per_s", "dof_updates_per_s", "latency_by_kind", "rate_req_per_s", "max_active",
            "rounds", "precision", "loop_seconds", "graph_steps", "group_streams")
    return {k: out[k] for k in keep}


def sweep_euler(sizes, steps=20):
    """Size sweep of the one-step Euler stage kernel (C0 physics, N_p = 2, 8 PEs, SAA) into the
    HBM-bound regime: per size, the stage kernel's mean launch time (HIP graphs, events over
    the timed steps) and its algorithmic bandwidth."""
    import torch

    from paper_2501_01747_amd import adg
    from workloads import gen

    import numpy as np

    out = []
    base_case, base = gen.case_c0(E=1024)
    for E in sizes:
        case, _ = gen.case_c0(E=min(E, 1024))
        case["disc"]["n_elem"] = E
        case["disc"]["dt"] *= min(E, 1024) / E      # same Courant number on the finer mesh
        # a smooth valid state of the right size: the 1024-element projection repeated
        w0 = np.ascontiguousarray(np.tile(base, (max(1, E // 1024), 1, 1))[:E]) if E >= 1024 else gen.case_c0(E=E)[1]
        s = adg.Solver(case)
        s.set_state(w0)
        s.step(3)
        ms = region_stage_ms(s, steps)
        nbytes = euler_stage_bytes(case)
        out.append({"n_elem": E, "dof": gen.dof(case), "stage_ms": ms, "GBps": nbytes / (ms * 1e-3) / 1e9,
                    "frac_hbm": nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "bytes": nbytes})
        s.close()
        del s
        torch.cuda.empty_cache()
    return out


def sweep_ns(sizes, steps=20):
    """Size sweep of the single-problem detailed-chemistry stage kernel: the ignition workload's
    physics at its element width (1 cm / 2048) and PE density (one PE per 128 elements), E
    elements (the 2048-element state repeated, a periodic domain of E/2048 cm), N_p = 3; per
    size the decomposition the autotuner keeps, the mean launch time (HIP events over
    graph-replayed steps) and the algorithmic FP64 rate against the 78.6 TFLOP/s peak."""
    import numpy as np
    import torch

    from paper_2501_01747_amd import adg
    from workloads import gen

    mech = gen.c1_mechanism()
    _, base = gen.case_c1(mech=mech)
    out = []
    for E in sizes:
        if E >= 2048:
            case, _ = gen.case_c1(E=2048, mech=mech, n_pe=16)
            case["disc"]["n_elem"] = E
            case["disc"]["x_right"] = case["disc"]["x_left"] + 0.01 * E / 2048
            case["async"]["n_pe"] = E // 128
            w0 = np.ascontiguousarray(np.tile(base, (E // 2048, 1, 1)))
        else:
            case, w0 = gen.case_c1(E=E, Lx=0.01 * E / 2048, n_pe=max(1, E // 128), mech=mech)
        s = adg.Solver(case)
        s.set_state(w0)
        cfg = s.autotune()
        s.set_state(w0)
        ms = region_stage_ms(s, steps)
        flops = detailed_stage_flops(case)
        try:
            s.sync()              # raises if the run latched a state error
            state_ok = True
        except Exception:
            state_ok = False
        out.append({"n_elem": E, "dof": gen.dof(case), "n_pe": case["async"]["n_pe"], "kernel_config": cfg,
                    "stage_ms": ms, "TFLOPs": flops / (ms * 1e-3) / 1e12,
                    "frac_fp64": flops / (ms * 1e-3) / 1e12 / FP64_VECTOR_PEAK_TFLOPS,
                    "steps": s.step_count(), "state_ok": state_ok})
        s.close()
        del s
        torch.cuda.empty_cache()
        print(json.dumps(out[-1]), flush=True)
    return out


def sweep_limiter(sizes, steps=20):
    """Size sweep of the one-step stage kernel with the limiter inside (the detonation
    workload's physics at its resolution dx = 1/32, N_p = 3, HLLC, KXRCF + AT-WENO, 64 PEs):
    per size, the kernel's mean launch time (as in sweep_euler) and its algorithmic bandwidth."""
    import torch

    from paper_2501_01747_amd import adg
    from workloads import gen

    out = []
    for E in sizes:
        case, w0 = gen.case_c2(E=E, length=E / 32.0, shock_x=E / 512.0)
        s = adg.Solver(case)
        s.set_state(w0)
        s.step(3)
        ms = region_stage_ms(s, steps)
        nbytes = euler_stage_bytes(case)
        out.append({"n_elem": E, "dof": gen.dof(case), "stage_ms": ms, "GBps": nbytes / (ms * 1e-3) / 1e9,
                    "frac_hbm": nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "bytes": nbytes})
        s.close()
        del s
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="c1")
    ap.add_argument("--graph", type=int, default=50, help="time steps per captured HIP graph (0 = plain launches)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-peaks", action="store_true", help="skip the measured copy / FP64 ceilings")
    ap.add_argument("--sweep-ns", action="store_true",
                    help="print the single-problem detailed-chemistry stage-kernel size sweep instead of the benchmark line")
    ap.add_argument("--sweep-euler", action="store_true",
                    help="print the one-step stage-kernel size sweeps (without and with the limiter) instead of the benchmark line")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="calibration copy + plain-launch steps for rocprofv3 --pmc (no benchmark line)")
    ap.add_argument("--n-elem", type=int, default=None, help="override the workload's element count")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched mixed-precision measurement")
    ap.add_argument("--batch-steps", type=int, default=60, help="timed steps of the batched workload")
    ap.add_argument("--precision", default="mixed", help="batched workload precision: mixed | fp64")
    ap.add_argument("--serve-graph", type=int, default=2,
                    help="served stream: steps per captured batch graph (0: plain launches)")
    ap.add_argument("--group-streams", type=int, default=None,
                    help="served stream: streams a stage's group launches are spread over (1..4; default 4)")
    ap.add_argument("--requests", type=int, default=1000, help="served stream: number of requests")
    ap.add_argument("--rate", type=float, default=None, help="served stream: arrival rate (requests/s)")
    ap.add_argument("--calibrate", action="store_true", help="served stream: saturation run (all arrive at t=0)")
    ap.add_argument("--serve-heap-gib", type=float, default=16.0)
    ap.add_argument("--serve-slots", type=int, default=1024)
    ap.add_argument("--serve-chunk", type=int, default=10)
    ap.add_argument("--served-requests", type=int, default=160,
                    help="default line: requests of the short served stream (0 = skip)")
    ap.add_argument("--no-hbm-points", action="store_true", help="default line: skip the HBM-bound Euler points")
    ap.add_argument("--batch-decompositions", action="store_true",
                    help="time every work decomposition of the batched kernel (no benchmark line)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(sharding across GPUs is designed, not built)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2501_01747_amd import adg
    from workloads import gen

    torch.cuda.set_device(0)
    if args.batch_decompositions:
        batch_decompositions(args.steps, args.precision)
        return
    if args.workload == "c3" and not args.pmc_probe:
        out = bench_batched(args.steps, args.warmup, args.graph, args.precision, cpu=not args.no_cpu_baseline)
        out.update({"metric": METRIC, "n_gpus": 1, "higher_is_better": True, "scaling": "weak",
                    "vs_baseline": None, "dtype": "f64+f32" if args.precision == "mixed" else "f64",
                    "data": "synthetic"})
        print(json.dumps(out), flush=True)
        return
    if args.workload == "c4":
        rate = None if args.calibrate else (args.rate or C4_RATE)
        if rate is None and not args.calibrate:
            raise SystemExit("no arrival rate: run with --calibrate first or pass --rate")
        out = bench_serve(args.requests, rate, args.serve_heap_gib, args.serve_slots, args.serve_chunk,
                          args.precision, args.group_streams, args.serve_graph)
        out.update({"metric": METRIC, "workload": "c4_served_stream", "n_gpus": 1, "data": "synthetic",
                    "saturation_run": bool(args.calibrate)})
        if args.calibrate:
            out["calibrated_rate_req_per_s"] = 0.7 * out["requests_per_s"]
        print(json.dumps(out), flush=True)
        return
    if args.pmc_probe:
        pmc_probe(args)
        return
    if args.sweep_ns:
        print(json.dumps({"sweep": "ns_stage_kernel", "results": sweep_ns([2**p for p in range(11, 21, 1)])}),
              flush=True)
        return
    if args.sweep_euler:
        print(json.dumps({"sweep": "euler_stage_kernel", "results": sweep_euler([2**p for p in range(10, 24, 1)])}),
              flush=True)
        print(json.dumps({"sweep": "euler_lim_kernel", "results": sweep_limiter([2**p for p in range(13, 23, 1)])}),
              flush=True)
        return
    case, w0 = workload(args.workload, args.n_elem)
    s = adg.Solver(case)
    s.set_state(w0)
    tuned = s.autotune()
    # graphs of min(--graph, K) steps: the timed K steps are K // g replays and K mod g plain
    # steps (the library keeps a graph for each step alignment, so none realigns)
    graph = min(args.graph, args.steps)
    if graph:
        s.set_graph(graph)
    s.step(max(args.warmup, 1))   # captures the graphs (the first step after set_graph)
    s.sync()
    replays0 = s.graph_replays
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(s.stream)
    s.step(args.steps)
    ev1.record(s.stream)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    s.sync()
    replays = s.graph_replays - replays0
    dof = gen.dof(case)
    value = dof * 3 * args.steps / el
    ms_per_step = el * 1e3 / args.steps

    # dominant kernel: the stage kernel, the only kernel of a step (one launch per RK stage):
    # its mean launch duration is the HIP-event time of the timed region on the solver's
    # stream over the launches in it
    stage_ms = ev0.elapsed_time(ev1) / (args.steps * RK_STAGES[case["disc"].get("rk", "ssprk3")])
    # each launch alone between its own pair of events (includes its dispatch), for reference
    prof = s.profile(max(10, min(args.steps, 50)))
    detailed = case["physics"]["model"] == "detailed"
    kernel_src = ["adg_ns.hip", "adg_ns.hpp"] if detailed else ["adg_euler.hip", "adg_device.hpp"]
    traffic_key = args.workload if args.n_elem is None else f"{args.workload}_{args.n_elem}"
    if detailed:
        flops = detailed_stage_flops(case)
        achieved = flops / (stage_ms * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP64_VECTOR_PEAK_TFLOPS, "traffic": read_traffic(traffic_key, kernel_src),
                "kernel": "ns_stage_kernel", "launch_ms": stage_ms, "flops_per_launch": flops}
    else:
        nbytes = euler_stage_bytes(case)
        achieved = nbytes / (stage_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": read_traffic(traffic_key, kernel_src),
                "kernel": "euler_lim_kernel" if case["disc"].get("limiter") else "euler_stage_kernel",
                "launch_ms": stage_ms, "bytes_per_launch": nbytes}
    d = case["disc"]
    out = {
        "metric": METRIC, "value": value, "unit": "DOF-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": case["name"], "n_elem": d["n_elem"], "order_p": d["order_p"],
                   "n_vars": 3 + case["physics"]["n_species"], "n_pe": case["async"]["n_pe"],
                   "delays": case["async"]["mode"], "dof": dof, "graph_steps": graph,
                   "timed_graph_replays": replays, "timed_plain_steps": args.steps - replays * graph,
                   "dt": d["dt"], "cfl": case.get("cfl"),
                   "dt_convention": "dt = CFL dx / ((2 N_p + 1) lambda_0), lambda_0 = max |u| + a of the initial state",
                   "kernel_config": tuned},
        "roofline": roof,
        "isolated_launch_ms": {k: v[0] for k, v in prof.items()},
    }
    s.close()
    if not args.no_peaks:
        # the device's measured ceilings (project-written copy and FP64 FMA kernels), beside
        # the published peaks the roofline fraction uses
        from paper_2501_01747_amd import peaks

        mp = peaks.measure()
        out["measured_peaks"] = mp
        ceiling = mp["fp64_vector_TFLOPs"] if detailed else mp["copy_GBps"]
        out["roofline"]["frac_of_measured"] = out["roofline"]["achieved"] / ceiling
    if not args.no_batched and detailed:
        bb = bench_batched(args.batch_steps, 5, args.graph, args.precision, cpu=not args.no_cpu_baseline)
        out["batched_mixed"] = bb
        out["batched_over_plain"] = bb["value"] / value
    if args.served_requests > 0 and detailed:
        out["served"] = served_short(args.served_requests, args.rate or C4_RATE, args.precision)
    if not args.no_hbm_points:
        out["hbm_points"] = hbm_points()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(case, w0)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
