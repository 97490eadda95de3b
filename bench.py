#!/usr/bin/env python
"""Benchmark of the GGArray hot path on one MI355X.

Workload (one step): configuration 2 of the project, the paper's doubling-growth
experiment at scale (Sec. VI-C) -- a GGArray of 512 LFVectors of uint32 with
first bucket 1024 receives 2^28 insertions over 12 growth rounds (n_0 = 2^17,
n_r = 2^(16+r)); after every round each LFVector pops a tenth of its elements
(shrink 1/10); then one r/w pass x = 3x + 1 over every live element; then the
prefix-sum flatten into a contiguous buffer.  Each step starts by emptying the
array (shrink 1/1): that clear, the twelve rounds and their shrinks are one
ggarray_insert_gen_rounds call, which runs them in one launch (each LFVector's
wave takes it through every round, taking the buckets it kept through the clear
again).  Payloads are generated on the device: thread gid of
round r inserts (r << 27) | gid.  All input is synthetic.

`value` is the step throughput in inserted elements per second (Gelem/s) with
nothing but the array metadata resident when the timed region starts.  Per-kernel
HIP-event timings give insert Gelem/s and r/w / flatten HBM GB/s; the static
array and the host-resized (semi-static) array run the same insertion rounds
and r/w pass beside it.  The CPU oracle runs the same workload on the host.

One JSON line is printed.  Only one GPU is used; --gpus above 1 is refused.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import statistics
import sys
import time
import traceback

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "insert Gelem/s + r/w HBM GB/s (vs static array); p50/p99 latency served"
HBM_PEAK_GBPS = 8000.0
F, ELEM, TAG_SHIFT = 1024, 4, 27


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--vectors", type=int, default=512, help="LFVectors (the paper's 32 / 512 sweep)")
    ap.add_argument("--no-baselines", action="store_true", help="skip static / semi-static arrays")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg and its parity check")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched (512-array) leg")
    ap.add_argument("--no-served", action="store_true", help="skip the served (4096-array request loop) leg")
    ap.add_argument("--no-two-phase", action="store_true", help="skip the growth-then-work case study")
    ap.add_argument("--no-config1", action="store_true", help="skip the small launch-bound (configuration 1) leg")
    ap.add_argument("--no-config3", action="store_true", help="skip the irregular-insertion (configuration 3) leg")
    ap.add_argument("--no-ceiling", action="store_true", help="skip the plain fill / copy rate measurement")
    ap.add_argument("--no-shootout", action="store_true",
                    help="skip the scan-vs-atomic insertion comparison and the memory model")
    ap.add_argument("--serve-requests", type=int, default=1 << 20, help="requests in the served trace")
    ap.add_argument("--serve-lanes", type=int, default=2,
                    help="served steps in flight (2 measured best: at 5.45e4 / 9.8e4 req/s p99 111 / 100 us "
                         "against 153 / 159 with 3 lanes and 176 / 182 with 1)")
    ap.add_argument("--serve-step", type=int, default=1024, help="requests per served step")
    ap.add_argument("--serve-baseline-requests", type=int, default=1 << 14,
                    help="trace prefix replayed with one launch per request")
    ap.add_argument("--traffic", default=TRAFFIC_SUMMARY,
                    help="rocprofv3 counter summary with measured HBM bytes per launch")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 2 GiB device copy (torch), to calibrate HBM byte counters")
    ap.add_argument("--batched-counters", action="store_true",
                    help="only run the configuration-4 batch with one launch per phase (for HBM byte counters)")
    return ap.parse_args()


def copy_calibration():
    """A plain copy kernel of known size: 2 GiB read, 2 GiB written, three times."""
    import torch
    torch.cuda.set_device(0)
    a = torch.empty(1 << 29, dtype=torch.int32, device="cuda").fill_(1)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": 2 * a.numel() * 4, "repeats": 3}), flush=True)


def batched_counters():
    """The configuration-4 batch alone, for hardware counters: first buckets from the
    capacity rule (no tuning), two passes of clear, 4 keyed rounds, r/w x + 1 and
    flatten with one launch per phase (no cooperative launch)."""
    import torch
    from paper_2209_00103_amd import autotune as at, ggarray as G, workloads as wl
    torch.cuda.set_device(0)
    sizes = [int(x) for x in wl.cfg4_sizes(1, 512)]
    vecs = [wl.cfg4_vectors(n) for n in sizes]
    firsts = []
    for n, V in zip(sizes, vecs):
        rounds = wl.cfg4_round_threads(n, 4)
        ok = [F for F in at.CANDIDATES if at.predicted_ratio(n, V, F, rounds) <= 2.0] or [at.CANDIDATES[0]]
        firsts.append(max(ok))
    total = sum(sizes)
    pool = G.Pool(int(4 * total * 2.2) + (256 << 20))
    arrays = [G.GGArray(pool, 4, V, F) for V, F in zip(vecs, firsts)]
    b = G.Batch(arrays)
    out = torch.empty(total, dtype=torch.int32, device="cuda")
    counts = [[wl.cfg4_round_threads(n, 4)[r] for n in sizes] for r in range(4)]
    gens = [G.make_gen(G.GEN_KEYED, seed=1, round=r, tag=0) for r in range(4)]
    for _ in range(2):
        b.shrink(1, 1)
        for r in range(4):
            b.insert_gen(gens[r], counts[r])
        b.rw(G.ADD1)
        b.flatten_into(out)
    torch.cuda.synchronize()
    assert b.last_error() == 0
    b.close()
    for a in arrays:
        a.close()
    pool.close()
    print(json.dumps({"batched_counters_elements": total, "passes": 2}), flush=True)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def stage(name):
    """A short progress mark on stderr as each leg starts (names the leg that was
    running if the process ends early)."""
    print(f"[{time.strftime('%H:%M:%S')}] {name}", file=sys.stderr, flush=True)


def ceiling_leg(torch, n_small=None, reps=10):
    """Achievable streaming rates on this GPU with plain PyTorch kernels over 4 GiB:
    a write-only fill, a copy (4 GiB read, 4 GiB written) and an in-place add (the
    same 4 GiB read and written, the access pattern of r/w); with n_small also the
    copy and the in-place add over n_small int32 words (the array's live size, so
    the same bytes as one r/w or flatten).  Context for the roofline fractions,
    which stay against the 8 TB/s specification."""
    n = 1 << 30  # int32 words: 4 GiB per buffer
    a = torch.empty(n, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)

    def rate(fn, moved):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        return {"GBps": moved / (ms * 1e-3) / 1e9, "ms": ms}

    res = {"fill": rate(lambda: a.fill_(7), 4 * n), "copy": rate(lambda: b.copy_(a), 8 * n),
           "inplace_add": rate(lambda: a.add_(1), 8 * n), "bytes_per_buffer": 4 * n,
           "note": "torch fill_, copy_ and add_ over 4 GiB int32 buffers; bytes moved per call / time"}
    if n_small:
        sa, sb = a[:n_small], b[:n_small]
        res["same_size"] = {"words": n_small, "copy": rate(lambda: sb.copy_(sa), 8 * n_small),
                            "inplace_add": rate(lambda: sa.add_(1), 8 * n_small)}
    del a, b
    torch.cuda.empty_cache()
    return res


TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "cfg2_hbm_traffic.md")
VALU_SUMMARY = os.path.join(ROOT, "profiles", "cfg3_insert_alu.md")


def kernel_source_digest() -> str:
    """Digest of the HIP sources and the device header, comments and blank space
    removed; a counter figure counts only if it was measured on the same code."""
    import hashlib
    import re
    csrc = os.path.join(ROOT, "paper_2209_00103_amd", "csrc")
    files = [os.path.join(csrc, n) for n in sorted(os.listdir(csrc)) if n.endswith((".hip", ".h"))]
    files.append(os.path.join(ROOT, "include", "ggarray_device.h"))
    h = hashlib.sha256()
    for path in files:
        with open(path) as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        text = " ".join(text.split())
        h.update(os.path.basename(path).encode() + b"\0" + text.encode())
    return h.hexdigest()[:16]


def measured_counter(path: str, key: str, kernel: str):
    """A per-launch counter figure of `kernel` from a rocprofv3 summary (its line
    `key: {json}`), or None when there is none or the kernels changed since."""
    if not path or not os.path.exists(path):
        return None
    with open(path) as f:
        for line in f:
            if line.startswith(key + ":"):
                d = json.loads(line.split(":", 1)[1])
                if d.get("digest") == kernel_source_digest():
                    return d.get(kernel)
    return None


def measured_traffic(path: str, kernel: str):
    """HBM bytes per launch of `kernel` from the rocprofv3 counter summary, or None
    when there is none or the kernels changed since it was taken."""
    return measured_counter(path, "traffic_bytes_per_launch", kernel)


class Timer:
    """HIP events on torch's current stream, the stream every library call uses."""

    def __init__(self, torch):
        self.torch = torch
        self.marks = {}

    def span(self, name):
        torch = self.torch
        t = self

        class _S:
            def __enter__(self):
                self.a = torch.cuda.Event(enable_timing=True)
                self.b = torch.cuda.Event(enable_timing=True)
                self.a.record()

            def __exit__(self, *exc):
                self.b.record()
                t.marks.setdefault(name, []).append((self.a, self.b))

        return _S()

    def ms(self, name):
        return [a.elapsed_time(b) for a, b in self.marks.get(name, [])]


def ggarray_step(G, arr, gens, rounds, out, prefix_buf, timer=None, round_ms=None):
    """One step: clear, 12 rounds with their shrinks, prefix, r/w, flatten.  The
    clear and the rounds run as one ggarray_insert_gen_rounds call (one launch;
    the clear keeps the buckets the rounds take again), except in the per-kernel
    pass (timer / round_ms given), which times each round as its own
    ggarray_insert_gen_shrink launch (the round, then its shrink 1/10) and the
    clear as its own shrink 1/1 at the end of the step."""
    def span(name):
        return timer.span(name) if timer else _Null()

    fused = timer is None and round_ms is None
    if fused:
        arr.insert_gen_rounds(gens, rounds, 1, 10, clear_first=True)
    else:
        for r, n in enumerate(rounds):
            with span(f"insert{r}"):
                arr.insert_gen_shrink(gens[r], n, 1, 10)
            if round_ms is not None:  # kernel timing on: the launch's own start / end events
                round_ms[r].append(arr.kernel_ms(2))
    with span("prefix"):
        arr.prefix_into(prefix_buf)
    with span("rw"):
        arr.rw(G.MUL3ADD1)
    with span("flatten"):
        arr.flatten_into(out)
    if not fused:
        with span("clear"):
            arr.shrink(1, 1)


class _Null:
    def __enter__(self):
        return self

    def __exit__(self, *exc):
        return False


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def _pct(xs, q):
    xs = sorted(xs)
    return xs[min(len(xs) - 1, int(round(q / 100.0 * (len(xs) - 1))))]


def batched_leg(G, wl, torch, np, steps, warmup):
    """Configuration 4: 512 arrays with log-uniform target sizes 2^10..2^24 (uint32),
    4 insertion rounds of ceil(n/4) threads each (keyed payloads), r/w x+1,
    flatten to per-array offsets.  One step = clear + 4 rounds + r/w + flatten.
    Timed as one launch per phase for all arrays (eager and replayed as a captured
    HIP graph) against one launch per array and phase (eager and captured).  The
    batched and per-array results must be identical; parity with the oracle at this
    size is a GPU test."""
    from paper_2209_00103_amd.autotune import AutoTuner

    n_arr = 512
    sizes = [int(x) for x in wl.cfg4_sizes(1, n_arr)]
    vecs = [wl.cfg4_vectors(n) for n in sizes]
    rounds = [wl.cfg4_round_threads(n, 4) for n in sizes]
    tuner = AutoTuner(wl.cfg4_vectors, lambda n: wl.cfg4_round_threads(n, 4), elem_bytes=ELEM)
    firsts = [tuner.first_bucket(n) for n in sizes]
    total = sum(sizes)
    pool = G.Pool(int(ELEM * total * 2.2) + (256 << 20))
    arrays = [G.GGArray(pool, ELEM, vecs[i], firsts[i]) for i in range(n_arr)]
    b = G.Batch(arrays)
    out = torch.empty(total, dtype=torch.int32, device="cuda")
    out2 = torch.empty(total, dtype=torch.int32, device="cuda")
    out3 = torch.empty(total, dtype=torch.int32, device="cuda")
    counts0 = [rounds[i][0] for i in range(n_arr)]
    b.insert_gen(G.make_gen(G.GEN_KEYED, seed=1, round=0, tag=0), counts0)  # something to stream while tuning
    grid = tuner.tune_grid(b, out, total)
    counts = [[rounds[i][r] for i in range(n_arr)] for r in range(4)]
    bgens = [G.make_gen(G.GEN_KEYED, seed=1, round=r, tag=0) for r in range(4)]
    agens = [[G.make_gen(G.GEN_KEYED, seed=1, round=r, tag=i) for r in range(4)] for i in range(n_arr)]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    views = [out2[int(offs[i]):int(offs[i + 1])] for i in range(n_arr)]

    def batched_step():
        b.shrink(1, 1)
        for r in range(4):
            b.insert_gen(bgens[r], counts[r])
        b.rw(G.ADD1)
        b.flatten_into(out)

    def persistent_step():  # the clear runs inside the step's launch
        b.step(bgens, counts, G.ADD1, out3, clear=True)

    def per_array_step():
        for i, a in enumerate(arrays):
            a.shrink(1, 1)
            for r in range(4):
                a.insert_gen(agens[i][r], rounds[i][r])
            a.rw(G.ADD1)
            a.flatten_into(views[i])

    def timed(fn, k):
        ts = []
        for _ in range(k):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return ts

    s = torch.cuda.Stream()
    res = {}
    with torch.cuda.stream(s):
        for _ in range(max(1, warmup)):
            batched_step()
        s.synchronize()
        res["batched"] = timed(batched_step, steps)
        for _ in range(max(1, warmup)):
            persistent_step()
        s.synchronize()
        res["persistent"] = timed(persistent_step, steps)
        per_array_step()  # warm-up (uploads nothing, sizes status buffers)
        s.synchronize()
        res["per_array"] = timed(per_array_step, max(2, min(steps, 3)))
    g1 = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g1, stream=s):
        batched_step()
    g2 = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g2, stream=s):
        per_array_step()
    g3 = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g3, stream=s):
        persistent_step()
    with torch.cuda.stream(s):
        g1.replay()
        g2.replay()
        g3.replay()
        s.synchronize()
        res["batched_graph"] = timed(g1.replay, steps)
        res["per_array_graph"] = timed(g2.replay, steps)
        res["persistent_graph"] = timed(g3.replay, steps)
    torch.cuda.synchronize()
    assert b.last_error() == 0
    got, got2 = G.as_unsigned(out), G.as_unsigned(out2)
    same = bool(np.array_equal(got, got2))
    same_persistent = bool(torch.equal(out, out3))
    cap = sum(a.capacity() for a in arrays)
    for a in arrays:
        a.close()
    b.close()
    pool.close()
    summary = {}
    for k, ts in res.items():
        summary[k] = {"mean_ms": statistics.mean(ts), "p50_ms": _pct(ts, 50), "p99_ms": _pct(ts, 99),
                      "Gelem_s": total / (statistics.mean(ts) * 1e-3) / 1e9}
    fhist = {}
    for F in firsts:
        fhist[str(F)] = fhist.get(str(F), 0) + 1
    return {"workload": "512 arrays, sizes log-uniform 2^10..2^24 uint32, 4 keyed insertion rounds, "
                        "r/w x+1, flatten to per-array offsets",
            "elements": total, "lfvectors": sum(vecs), "timings": summary,
            "capacity_over_live": cap / total, "first_bucket_choices": fhist, "stream_grid": grid,
            "batched_equals_per_array": same, "persistent_equals_batched": same_persistent}


def _latency(res, arrival, kind, k):
    lat = (res["t_done_ns"][:k].astype(np.int64) - arrival[:k].astype(np.int64)) / 1e3
    ok = res["status"][:k] == 0
    out = {}
    for name, sel in (("all", ok), ("append", ok & (kind[:k] == 0)), ("rw", ok & (kind[:k] == 1)),
                      ("flatten", ok & (kind[:k] == 2))):
        x = lat[sel]
        out[name] = {"n": int(x.size), "p50_us": float(np.percentile(x, 50)) if x.size else None,
                     "p99_us": float(np.percentile(x, 99)) if x.size else None,
                     "mean_us": float(x.mean()) if x.size else None}
    return out


def served_leg(G, wl, torch, np_, args):
    """Configuration 5: 4096 resident arrays (initial sizes lognormal, median 2^16
    uint32, sigma 1), a trace of 2^20 requests (60% append of lognormal length with
    median 2^10, 30% r/w x+1, 10% flatten; uniform targets; exponential gaps), a
    64 GiB admission budget.  First the saturation throughput (every request queued
    at t = 0), then offered loads of 0.25 .. 1.1 x saturation with latency
    percentiles per request type.  Baseline: one launch per request, in arrival
    order, on a prefix of the same trace at the same offered rate.  Every run starts
    from the same resident state."""
    cfg = wl.CFG5
    seed, n_arr, n = 1, cfg["n_arrays"], int(args.serve_requests)
    sizes = [int(x) for x in wl.cfg5_sizes(seed, n_arr, cfg["median_log2"], cfg["sigma"], cfg["size_cap_log2"])]
    vecs = [wl.cfg4_vectors(s) for s in sizes]
    firsts = [wl.cfg5_first_bucket(s, v) for s, v in zip(sizes, vecs)]
    tr = wl.cfg5_trace(seed, n, n_arr, cfg["append_median_log2"], cfg["append_cap_log2"], cfg["mix"])
    kind, target, length = tr["kind"], tr["target"], tr["length"]
    final_live = sum(sizes) + int(length.sum())
    pool = G.Pool(ELEM * (2 * final_live + sum(v * f for v, f in zip(vecs, firsts))) + (1 << 30))
    arrays = [G.GGArray(pool, ELEM, v, f) for v, f in zip(vecs, firsts)]
    fill = G.Batch(arrays)
    fill_gen = G.make_gen(G.GEN_KEYED, seed=seed, round=cfg["fill_round"], tag=0)
    arena = torch.empty((4 << 30) // 4, dtype=torch.int32, device="cuda")
    out_len = torch.empty(n, dtype=torch.int64, device="cuda")
    common = dict(seed=seed, append_round=cfg["append_round"], append_shift=cfg["append_shift"], rw_op=G.ADD1)
    batched = G.Server(arrays, arena, cfg["cap_bytes"], mode=G.SERVE_BATCHED, lanes=args.serve_lanes,
                       max_step=args.serve_step, **common)
    per_req = G.Server(arrays, arena, cfg["cap_bytes"], mode=G.SERVE_PER_REQUEST, depth=1024, **common)

    def run(sv, arrival, k):
        fill.shrink(1, 1)  # back to the initial state: empty, buckets released, refilled
        fill.insert_gen(fill_gen, sizes)
        torch.cuda.synchronize()
        res = sv.run(arrival[:k], kind[:k], target[:k], length[:k], out_len)
        span = max(int(res["t_done_ns"][:k].max()), 1)
        done = res["status"][:k] == 0
        elems = int(length[:k][done & (kind[:k] == 0)].sum())
        return {"requests": k, "req_per_s": k / (span * 1e-9), "span_ms": span / 1e6,
                "appended_elems": elems, "rejected": res["rejected"], "steps": res["steps"],
                "mean_step": res["issued"] / max(res["steps"], 1), "largest_step": res["largest_step"],
                "memory_waits": res["memory_waits"], "peak_charged_GB": res["peak_charged_bytes"] / 1e9,
                "arena_wraps": res["arena_wraps"], **_latency(res, arrival, kind, k)}

    zeros = np_.zeros(n, dtype=np_.uint64)
    sat = run(batched, zeros, n)
    k_b = min(n, int(args.serve_baseline_requests))
    sat_pr = run(per_req, zeros, k_b)
    x = sat["req_per_s"]
    # loads the per-request baseline can sustain: 0.5 and 0.9 of its own saturation
    # rate, both modes on the same requests.  Tail latency at these light loads
    # varies from run to run on the same box (host and clock noise: the same build
    # has given p99 50 us and 124 us in consecutive processes), so each mode is
    # replayed three times, alternating, and the trial with the median p99 is
    # reported, all three p99s beside it.
    def median_trial(trials):
        order = sorted(range(len(trials)), key=lambda i: trials[i]["all"]["p99_us"])
        best = dict(trials[order[len(order) // 2]])
        best["trials_p99_us"] = [t["all"]["p99_us"] for t in trials]
        return best

    matched = []
    for f in (0.5, 0.9):
        rate = f * sat_pr["req_per_s"]
        arrival = wl.cfg5_arrivals_ns(tr["gap"], rate)
        tb, tp = [], []
        for _ in range(3):
            tb.append(run(batched, arrival, k_b))
            tp.append(run(per_req, arrival, k_b))
        m = {"load_of_per_request_saturation": f, "offered_req_per_s": rate,
             "batched": median_trial(tb), "per_request": median_trial(tp)}
        matched.append(m)
        log(f"served at {rate:.3e} req/s: batched p50 {m['batched']['all']['p50_us']:.0f} us p99 "
            f"{m['batched']['all']['p99_us']:.0f} us (trials {[round(x) for x in m['batched']['trials_p99_us']]}); "
            f"per-request p50 {m['per_request']['all']['p50_us']:.0f} us "
            f"p99 {m['per_request']['all']['p99_us']:.0f} us (trials {[round(x) for x in m['per_request']['trials_p99_us']]})")
    loads = []
    for f in cfg["loads"]:
        arrival = wl.cfg5_arrivals_ns(tr["gap"], f * x)
        b = run(batched, arrival, n)
        b_prefix = run(batched, arrival, k_b)
        p = run(per_req, arrival, k_b)
        loads.append({"load": f, "offered_req_per_s": f * x, "batched": b,
                      "batched_prefix": {key: b_prefix[key] for key in ("req_per_s", "all", "append", "rw", "flatten")},
                      "per_request": p})
    batched.close()
    per_req.close()
    fill.close()
    for a in arrays:
        a.close()
    pool.close()
    return {"workload": f"{n_arr} resident arrays, initial sizes lognormal (median 2^16 uint32, sigma 1), "
                        f"{n} requests: 60% append (lognormal length, median 2^10), 30% r/w x+1, "
                        f"10% flatten; uniform targets; Poisson arrivals; 64 GiB admission budget",
            "resident_initial_GB": ELEM * sum(sizes) / 1e9, "appended_GB": ELEM * int(length.sum()) / 1e9,
            "lanes": args.serve_lanes, "max_step": args.serve_step,
            "baseline": f"one launch per request, in order, on the first {k_b} requests, at most 1024 in flight",
            "saturation": sat, "saturation_per_request": sat_pr, "matched": matched, "loads": loads}


def mapped_baseline(G, torch, gens, rounds, steps):
    """The mapped (memMap) array on the configuration-2 rounds (no shrink) and r/w."""
    map_ins, map_rw, maps = [], [], 0
    for rep in range(max(2, min(steps, 3)) + 1):
        mp = G.MappedArray(ELEM, 1 << 28)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for r, n in enumerate(rounds):
            mp.insert_gen(gens[r], n)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        mp.rw(G.MUL3ADD1)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if rep > 0:
            map_ins.append(t1 - t0)
            map_rw.append(t2 - t1)
        maps = mp.maps()
        assert mp.size() == 1 << 28
        mp.close()
    return {"insert_Gelem_s": (1 << 28) / statistics.mean(map_ins) / 1e9,
            "rw_GBps": 2 * ELEM * (1 << 28) / statistics.mean(map_rw) / 1e9,
            "maps": maps, "timing": "host wall clock (growth synchronises)"}


def sparse_leg(G, torch, rounds, V, steps, warmup):
    """The configuration-2 round sizes with Bernoulli(1/2) insertion instead of
    every thread inserting: the GGArray takes its scan path (wave ballot, per-
    LFVector tickets and decoupled look-back, Sec. III-B), the static array one
    atomic per tile of 4096 threads.  Per round: inserted elements (4 B written
    each) over the device time of the insertion call."""
    gens = [G.make_gen(G.GEN_BERNOULLI, seed=1, round=r) for r in range(len(rounds))]
    pool = G.Pool(8 << 30)
    arr = G.GGArray(pool, ELEM, V, F)
    added, prev = [], 0
    for r, n in enumerate(rounds):  # sizing pass: elements each round inserts
        arr.insert_gen(gens[r], n)
        s1 = arr.size()
        added.append(s1 - prev)
        arr.shrink(1, 10)
        prev = arr.size()
    arr.shrink(1, 1)
    st = G.StaticArray(1 << 28, ELEM)
    res = {}
    for name in ("ggarray", "static"):
        tm = Timer(torch)
        for rep in range(warmup + steps):
            t = tm if rep >= warmup else Timer(torch)
            for r, n in enumerate(rounds):
                with t.span(f"r{r}"):
                    if name == "ggarray":
                        arr.insert_gen(gens[r], n)
                    else:
                        st.insert_gen(gens[r], n)
                if name == "ggarray":
                    arr.shrink(1, 10)
            if name == "ggarray":
                arr.shrink(1, 1)
            else:
                st.clear()
        torch.cuda.synchronize()
        ms = [statistics.median(tm.ms(f"r{r}")) for r in range(len(rounds))]
        res[name] = {"per_round_us": [round(1e3 * x, 2) for x in ms],
                     "per_round_GBps": [round(ELEM * a / (x * 1e-3) / 1e9, 1) for a, x in zip(added, ms)],
                     "Gelem_s": sum(added) / (sum(ms) * 1e-3) / 1e9,
                     "last_round_GBps": ELEM * added[-1] / (ms[-1] * 1e-3) / 1e9}
    # The same round sizes as prepared buffers (uint32 values, one flag byte per
    # thread set with probability 1/2, drawn untimed): the scan and look-back path
    # then reads 5 B per thread and writes 4 B per inserted element, an HBM-scale
    # figure for it.
    gen_t = torch.Generator(device="cuda")
    gen_t.manual_seed(7)
    bufs = []
    for n in rounds:
        vals = torch.randint(-(1 << 31), 1 << 31, (n,), dtype=torch.int32, device="cuda", generator=gen_t)
        flags = (torch.rand(n, device="cuda", generator=gen_t) < 0.5).to(torch.uint8)
        bufs.append((vals, flags, int(flags.sum())))
    for name in ("ggarray", "static"):
        tm = Timer(torch)
        for rep in range(warmup + steps):
            t = tm if rep >= warmup else Timer(torch)
            for r, (vals, flags, _) in enumerate(bufs):
                with t.span(f"r{r}"):
                    (arr if name == "ggarray" else st).insert(vals, flags)
                if name == "ggarray":
                    arr.shrink(1, 10)
            if name == "ggarray":
                arr.shrink(1, 1)
            else:
                st.clear()
        torch.cuda.synchronize()
        ms = [statistics.median(tm.ms(f"r{r}")) for r in range(len(rounds))]
        byt = [5 * n + ELEM * b[2] for n, b in zip(rounds, bufs)]
        res[name + "_buffer"] = {"per_round_us": [round(1e3 * x, 2) for x in ms],
                                 "per_round_GBps": [round(y / (x * 1e-3) / 1e9, 1) for y, x in zip(byt, ms)],
                                 "Gelem_s": sum(b[2] for b in bufs) / (sum(ms) * 1e-3) / 1e9,
                                 "last_round_GBps": byt[-1] / (ms[-1] * 1e-3) / 1e9,
                                 "last_round_frac": byt[-1] / (ms[-1] * 1e-3) / 1e9 / HBM_PEAK_GBPS}
    assert arr.last_error() == 0 and st.last_error() == 0
    del bufs
    st.close()
    arr.close()
    pool.close()
    res["buffer_bytes"] = "read 4 B value + 1 B flag per thread, write 4 B per inserted element"
    res["inserted_per_round"] = added
    res["insert_vs_static"] = res["ggarray"]["Gelem_s"] / res["static"]["Gelem_s"]
    res["workload"] = ("configuration-2 round sizes (2^17, 2^17 .. 2^27 threads), each thread inserting "
                       "K(1,gid,r) with probability 1/2; GGArray V = 512 (shrink 1/10 after each round, untimed) "
                       "against the static array (one atomic per 4096-thread tile)")
    return res


def two_phase_leg(G, torch, V, ms=(1, 3, 10), ks=(1, 10, 100, 1000), iters=5, final=10**9):
    """The two-phase application of Sec. VI-D: `iters` repetitions of a growth
    phase, in which each of the s live elements' threads inserts m more (m rounds of
    s threads, round-tag payloads), followed by a work phase of k passes of x + 1
    over every element.  The starting size is final / (1 + m)^iters, so every m
    ends at `final` uint32.  Three ways, each timed by device events around the
    whole pattern: (a) the GGArray grows, is flattened into a flat buffer, and the
    work runs there; (b) the work runs on the GGArray itself (its own r/w); (c) the
    mapped array grows (host-driven mapping, which synchronises) and the work runs
    on it.  (a) and (c) use the same work kernel (the flat-array r/w); the host
    time (c) spends mapping is reported beside it."""
    out = {}
    pool = G.Pool(10 << 30)
    arr = G.GGArray(pool, ELEM, V, F)
    flat_buf = torch.empty(final, dtype=torch.int32, device="cuda")
    flat = G.StaticArray(final, ELEM, buf=flat_buf)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    tag = 24  # round-tag payloads (round << 24) | gid; gid < 2^24 is not needed for timing

    def sizes_for(m):
        s0 = max(1, round(final / (1 + m) ** iters))
        return s0, [s0 * (1 + m) ** i for i in range(iters)]

    def grow_gg(m, s_before, r0):
        for j in range(m):
            arr.insert_gen(G.make_gen(G.GEN_ROUND_TAG, round=(r0 + j) & 0xFF, tag_shift=tag), s_before)

    rows = {}
    for m in ms:
        s0, starts = sizes_for(m)
        for k in ks:
            row = {}
            for mode in ("flatten_then_work", "ggarray_work"):
                arr.shrink(1, 1)
                arr.insert_gen(G.make_gen(G.GEN_ROUND_TAG, round=0, tag_shift=tag), s0)
                torch.cuda.synchronize()
                e0.record()
                for it, s_before in enumerate(starts):
                    grow_gg(m, s_before, 1 + it * m)
                    if mode == "flatten_then_work":
                        n_live = s_before * (1 + m)
                        arr.flatten_into(flat_buf[:n_live])
                        flat.set_size(n_live)
                        for _ in range(k):
                            flat.rw(G.ADD1)
                    else:
                        for _ in range(k):
                            arr.rw(G.ADD1)
                e1.record()
                torch.cuda.synchronize()
                row[mode + "_ms"] = e0.elapsed_time(e1)
            assert arr.last_error() == 0 and arr.size() == starts[-1] * (1 + m)
            mp = G.MappedArray(ELEM, final + (final >> 4))
            mp.insert_gen(G.make_gen(G.GEN_ROUND_TAG, round=0, tag_shift=tag), s0)
            torch.cuda.synchronize()
            map_host = 0.0
            e0.record()
            t_all = time.perf_counter()
            for it, s_before in enumerate(starts):
                for j in range(m):
                    t = time.perf_counter()
                    mp.insert_gen(G.make_gen(G.GEN_ROUND_TAG, round=(1 + it * m + j) & 0xFF, tag_shift=tag),
                                  s_before)
                    map_host += time.perf_counter() - t
                for _ in range(k):
                    mp.rw(G.ADD1)
            e1.record()
            torch.cuda.synchronize()
            row["mapped_ms"] = e0.elapsed_time(e1)
            row["mapped_wall_ms"] = (time.perf_counter() - t_all) * 1e3
            row["mapped_insert_host_ms"] = map_host * 1e3
            row["mapped_maps"] = mp.maps()
            assert mp.size() == starts[-1] * (1 + m)
            mp.close()
            row["speedup_flatten_vs_mapped"] = row["mapped_ms"] / row["flatten_then_work_ms"]
            row["speedup_ggarray_vs_mapped"] = row["mapped_ms"] / row["ggarray_work_ms"]
            rows[f"m{m}_k{k}"] = row
        out[str(m)] = {"start_size": s0, "final_size": starts[-1] * (1 + m)}
    flat.close()
    arr.close()
    pool.close()
    return {"workload": f"{iters} repetitions of (growth: each live element's thread inserts m more, "
                        f"m in {list(ms)}; work: k passes of x + 1), final size {final} uint32, "
                        f"GGArray V = {V}, F = {F}",
            "sizes": out, "rows": rows,
            "timing": "device events around the whole pattern on every side; (c)'s growth synchronises the host "
                      "(mapping), its host time inside the insert calls is mapped_insert_host_ms",
            "work_kernel": "(a) and (c): the flat-array r/w (one workgroup per 16 KiB tile); (b): the GGArray r/w"}


def shootout_leg(G, torch, reps=3):
    """The insertion-strategy comparison of Sec. VI-A on the static array: the
    block scan (one atomic per tile of 4096 threads) against one atomic per
    inserted element, for 2^20 .. 2^30 threads (10 doublings), every thread
    inserting with probability 1/2 (generated payloads)."""
    st = G.StaticArray(1 << 30, ELEM)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    rows = []
    for k in range(11):
        n = 1 << (20 + k)
        row = {"threads": n}
        for name, call in (("scan", st.insert_gen), ("atomic", st.insert_gen_atomic)):
            ts = []
            for rep in range(reps + 1):
                st.clear()
                g = G.make_gen(G.GEN_BERNOULLI, seed=1, round=rep)
                torch.cuda.synchronize()
                e0.record()
                call(g, n)
                e1.record()
                torch.cuda.synchronize()
                if rep:
                    ts.append(e0.elapsed_time(e1))
            row[name + "_us"] = 1e3 * statistics.median(ts)
            row[name + "_Gthreads_s"] = n / (statistics.median(ts) * 1e-3) / 1e9
        assert st.last_error() == 0
        row["scan_speedup"] = row["atomic_us"] / row["scan_us"]
        rows.append(row)
    st.close()
    return {"workload": "static array, 2^20..2^30 threads, each inserting K(1,gid,r) with probability 1/2",
            "rows": rows}


def memory_model_leg(G, torch, np_, N=1 << 20, V=512, samples=1000):
    """The memory comparison of Sec. V (Fig. 3), measured: a workload inserts
    N * LogNormal(0, sigma) elements.  A static array must be sized in advance;
    sized to fail at most 1% of the time it holds N * e^(2.326 sigma).  The
    GGArray is grown to each drawn size and its capacity read back; its first
    bucket is picked by the capacity bound (C <= 2S + V(F - 1) per array): the
    largest power of two with V * F <= N / 64, so the per-LFVector rounding stays
    small against the live data, as it does for Fig. 3's large arrays.  Reported
    per sigma over `samples` draws: mean and largest allocated / live for both."""
    rng = np_.random.default_rng(1)
    Fm = 1
    while V * Fm * 2 <= N // 64:
        Fm *= 2
    pool = G.Pool(16 << 30)
    a = G.GGArray(pool, ELEM, V, Fm)
    rows = []
    z99 = 2.3263478740408408
    cap_max = 1 << 30  # draws are clamped here, so that twice the live data fits the 16 GiB pool
    for sigma in [0.0, 0.25, 0.5, 0.75, 1.0, 1.25, 1.5, 1.75, 2.0]:
        x = np_.maximum(1, np_.rint(N * np_.exp(sigma * rng.standard_normal(samples)))).astype(np_.int64)
        x = np_.minimum(x, cap_max)
        static_cap = N * float(np_.exp(z99 * sigma))
        gg_ratio = []
        for n in x:
            a.insert_gen(G.make_gen(G.GEN_ROUND_TAG, round=0, tag_shift=40), int(n))
            gg_ratio.append(a.capacity() / int(n))
            a.shrink(1, 1)  # back to empty: every bucket returns to the pool
        st_ratio = static_cap / x
        rows.append({"sigma": sigma,
                     "ggarray_capacity_over_live": float(np_.mean(gg_ratio)),
                     "ggarray_capacity_over_live_max": float(np_.max(gg_ratio)),
                     "static_1pct_capacity_over_live": float(np_.mean(st_ratio[x <= static_cap])),
                     "static_fits_fraction": float(np_.mean(x <= static_cap))})
    assert a.last_error() == 0
    a.close()
    pool.close()
    return {"workload": f"N = {N}, {samples} draws per sigma (clamped at 2^30), GGArray V = {V}, "
                        f"F = {Fm} (V*F <= N/64)",
            "rows": rows}


def config1_leg(G, wl, torch, reps=200, warm=100):
    """Configuration 1 (small, launch-bound, cache-resident): 256 LFVectors, first
    bucket 1024, uint32, 2^18 threads per round inserting K(1, gid, r) with
    probability 1/2 over 4 rounds, r/w x + 1, flatten (about 2 MiB live).  Reported
    as latency: per-operation device time (HIP events; median and p10/p90 over
    `reps` steps) and the whole step eager and replayed as a HIP graph.  Each
    variant first runs `warm` untimed steps: the step is tens of microseconds, and
    a short burst after another leg measured 30-46 us for the same graph."""
    cfg = wl.CFG1
    pool = G.Pool(256 << 20)
    a = G.GGArray(pool, 4, cfg["V"], cfg["F"])
    gens = [G.make_gen(G.GEN_BERNOULLI, seed=1, round=r) for r in range(cfg["rounds"])]
    n = cfg["n_threads"]
    for g in gens:
        a.insert_gen(g, n)
    size = a.size()
    out = torch.empty(size, dtype=torch.int32, device="cuda")

    def step(t=None):
        a.shrink(1, 1)
        for r, g in enumerate(gens):
            with (t.span(f"insert{r}") if t else _Null()):
                a.insert_gen(g, n)
        with (t.span("rw") if t else _Null()):
            a.rw(G.ADD1)
        with (t.span("flatten") if t else _Null()):
            a.flatten_into(out)

    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        for _ in range(warm):
            step()
        timer = Timer(torch)
        for _ in range(reps):
            step(timer)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            step()
        e1.record()
    s.synchronize()
    eager_us = 1e3 * e0.elapsed_time(e1) / reps
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        step()
    for _ in range(warm):
        g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    graph_us = 1e3 * e0.elapsed_time(e1) / reps
    assert a.last_error() == 0 and a.size() == size
    ref = out.clone()

    # The same step as one persistent launch (gga_batch_step_clear on a batch of
    # this one array: every LFVector's clear, 4 rounds and r/w in one workgroup,
    # then the flatten), eager and replayed as a graph; its output must equal the
    # above.
    b = G.Batch([a])
    rows = [[n]] * len(gens)

    def pstep():  # the clear runs inside the step's launch
        b.step(gens, rows, G.ADD1, out, clear=True)

    with torch.cuda.stream(s):
        for _ in range(warm):
            pstep()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            pstep()
        e1.record()
    s.synchronize()
    p_eager_us = 1e3 * e0.elapsed_time(e1) / reps
    same = bool(torch.equal(out, ref))
    g2 = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g2, stream=s):
        pstep()
    for _ in range(warm):
        g2.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        g2.replay()
    e1.record()
    torch.cuda.synchronize()
    p_graph_us = 1e3 * e0.elapsed_time(e1) / reps
    same = same and bool(torch.equal(out, ref))
    assert a.last_error() == 0 and b.last_error() == 0
    b.close()
    a.close()
    pool.close()

    def pct(xs):
        q = sorted(xs)
        return {"p10_us": round(1e3 * q[int(0.1 * (len(q) - 1))], 2), "p50_us": round(1e3 * statistics.median(q), 2),
                "p90_us": round(1e3 * q[int(round(0.9 * (len(q) - 1)))], 2)}

    ops = {f"insert{r}": pct(timer.ms(f"insert{r}")) for r in range(len(gens))}
    ops["rw"] = pct(timer.ms("rw"))
    ops["flatten"] = pct(timer.ms("flatten"))
    return {"workload": "256 LFVectors, first bucket 1024, uint32, 4 rounds of 2^18 threads inserting "
                        "K(1,gid,r) with probability 1/2, r/w x+1, flatten", "final_size": size,
            "ops": ops, "step_us_eager": eager_us, "step_us_graph": graph_us, "reps": reps,
            "persistent_step": {"us_eager": p_eager_us, "us_graph": p_graph_us, "identical": same,
                                "what": "clear + gga_batch_step (4 rounds, r/w, flatten in one launch)"}}


def config3_leg(G, wl, torch, steps=3, pool_gib=24, close_gen_first=True):
    """Configuration 3 at full size (irregular insertion): uint64, V = 65536,
    F = 1024, 2^26 threads with Poisson(3) counts capped at 16 (thresholds from the
    host), 4 insert phases each followed by r/w x + 1, then flatten.  Device time
    per phase (HIP events), median over `steps` passes from an empty array.

    Two producers: gen mode (counts and payloads computed inside the insertion
    kernel, which makes it bound by vector-ALU issue) and buffer mode, where the
    same counts and payloads are prepared beforehand (untimed) and the round reads
    them: counts from the host generator, payloads packed in thread order (the
    flatten of one generated round into an empty array).  The two must give
    identical arrays; buffer mode is the HBM-bound insertion roofline."""
    thr = wl.poisson_thresholds(3, 16)
    n, V = 1 << 26, 65536
    # Both arrays of the leg (about 7.9 GB of buckets each) fit the pool together;
    # the generated-payload array is closed before the buffer-mode one is built.
    pool = G.Pool(pool_gib << 30)
    a = G.GGArray(pool, 8, V, 1024)
    gens = [G.make_gen(G.GEN_POISSON, seed=1, round=i, max_count=16, thresholds=thr) for i in range(4)]
    sizes = []
    for i in range(4):  # sizing pass
        a.insert_gen(gens[i], n)
        a.rw(G.ADD1)
        sizes.append(a.size())
    out = torch.empty(sizes[-1], dtype=torch.int64, device="cuda")
    a.shrink(1, 1)
    timer = Timer(torch)
    for rep in range(steps + 1):
        t = timer if rep else Timer(torch)
        for i in range(4):
            with t.span(f"ins{i}"):
                a.insert_gen(gens[i], n)
            with t.span(f"rw{i}"):
                a.rw(G.ADD1)
        with t.span("flatten"):
            a.flatten_into(out)
        if rep < steps:
            a.shrink(1, 1)
    torch.cuda.synchronize()
    assert a.last_error() == 0, f"generated rounds: device error {a.last_error()}"
    if close_gen_first:
        a.close()

    # Buffer mode: the same rounds as prepared inputs.
    pool2 = G.Pool(8 << 30)
    scratch = G.GGArray(pool2, 8, V, 1024)
    counts, packed = [], []
    for i in range(4):
        scratch.insert_gen(gens[i], n)
        packed.append(scratch.flatten())
        scratch.shrink(1, 1)
        counts.append(torch.from_numpy(wl.poisson_counts(1, i, n, thr)).to("cuda"))
        assert int(counts[-1].sum()) == packed[-1].numel(), "host counts differ from the generated round"
    scratch.close()
    pool2.close()
    b = G.GGArray(pool, 8, V, 1024)
    out_b = torch.empty(sizes[-1], dtype=torch.int64, device="cuda")
    tb = Timer(torch)
    for rep in range(steps + 1):
        t = tb if rep else Timer(torch)
        for i in range(4):
            with t.span(f"ins{i}"):
                b.insert_packed(packed[i], counts[i])
            with t.span(f"rw{i}"):
                b.rw(G.ADD1)
        with t.span("flatten"):
            b.flatten_into(out_b)
        if rep < steps:
            b.shrink(1, 1)
    torch.cuda.synchronize()
    assert b.last_error() == 0, f"buffer-mode rounds: device error {b.last_error()}"
    identical = bool(torch.equal(out, out_b))
    b.close()
    a.close()
    del packed, counts, out, out_b
    pool.close()

    def phases_of(tm, with_rw=True):
        prev, ph = 0, []
        for i in range(4):
            ins = statistics.median(tm.ms(f"ins{i}"))
            rw = statistics.median(tm.ms(f"rw{i}"))
            added = sizes[i] - prev
            prev = sizes[i]
            ph.append({"inserted": added, "insert_us": 1e3 * ins, "insert_Gelem_s": added / (ins * 1e-3) / 1e9,
                       "insert_GBps": 8 * added / (ins * 1e-3) / 1e9, "rw_us": 1e3 * rw,
                       "rw_GBps": 16 * sizes[i] / (rw * 1e-3) / 1e9})
        return ph

    phases = phases_of(timer)
    bphases = phases_of(tb)
    for p in bphases:  # algorithmic bytes of a buffer round: counts + payloads read, payloads written
        p["insert_bytes"] = n + 16 * p["inserted"]
        p["insert_traffic_GBps"] = p["insert_bytes"] / (p["insert_us"] * 1e-6) / 1e9
    fl = statistics.median(timer.ms("flatten"))
    # The generated insertion is bound by vector-ALU issue (SplitMix64 per element):
    # its roofline is the VALU instruction rate, from the committed counter summary
    # (VALU wave instructions per launch, valid while the kernel sources are
    # unchanged) over the live launch time, against 256 CUs x 4 SIMDs x 16 lanes x
    # 2.4 GHz.
    ins_us = statistics.median(p["insert_us"] for p in phases)
    valu = measured_counter(VALU_SUMMARY, "valu_per_launch", "insert")
    peak = 256 * 4 * 16 * 2.4e9 / 1e12
    roof = {"kernel": "insert_count_kernel (Poisson counts)", "bound": "alu", "unit": "T lane-instr/s",
            "peak": peak, "achieved": None, "frac": None, "valu_insts_per_launch": valu, "avg_launch_us": ins_us}
    if valu:
        roof["achieved"] = valu * 64 / (ins_us * 1e-6) / 1e12
        roof["frac"] = roof["achieved"] / peak
    sweep = config3_v_sweep(G, torch, gens, n, sizes[-1], steps)
    bus = statistics.median(p["insert_us"] for p in bphases)
    bbytes = statistics.mean(p["insert_bytes"] for p in bphases)
    broof = {"kernel": "insert_packed (tile sums + tile scan + insert_packed_kernel, one call)", "bound": "hbm",
             "unit": "GB/s", "peak": HBM_PEAK_GBPS, "bytes_per_call": bbytes, "avg_call_us": bus,
             "achieved": bbytes / (bus * 1e-6) / 1e9, "frac": bbytes / (bus * 1e-6) / 1e9 / HBM_PEAK_GBPS,
             "timing": "events around the call (its three launches)"}
    return {"workload": "2^26 threads, Poisson(3) counts capped at 16, uint64 K(1,gid,16i+j), V = 65536, "
                        "4 x (insert, r/w x+1), flatten", "final_size": sizes[-1], "phases": phases,
            "flatten_us": 1e3 * fl, "flatten_GBps": 16 * sizes[-1] / (fl * 1e-3) / 1e9, "insert_roofline": roof,
            "v_sweep": sweep,
            "buffer_mode": {"phases": bphases, "insert_roofline": broof, "identical_to_gen_mode": identical,
                            "inputs": "counts from the host generator, payloads packed in thread order "
                                      "(prepared before the timed passes)"}}


def config3_v_sweep(G, torch, gens, n, final_size, steps, vs=(512, 4096)):
    """Configuration 3's generated rounds with fewer LFVectors: V = 512 gives each
    LFVector 128 tiles of 1024 threads per round (tickets and the decoupled
    look-back at scale), V = 4096 gives 16.  Same 4 x (insert, r/w x + 1) passes;
    V changes the order of the elements but not the total, which is checked."""
    rows = []
    for V in vs:
        pool = G.Pool(16 << 30)
        a = G.GGArray(pool, 8, V, 1024)
        tm = Timer(torch)
        sizes = []
        for rep in range(steps + 1):
            t = tm if rep else Timer(torch)
            sizes = []
            for i in range(4):
                with t.span(f"ins{i}"):
                    a.insert_gen(gens[i], n)
                with t.span(f"rw{i}"):
                    a.rw(G.ADD1)
                if rep == 0:
                    sizes.append(a.size())
            if rep == 0:
                first_sizes = sizes
            if rep < steps:
                a.shrink(1, 1)
        torch.cuda.synchronize()
        assert a.last_error() == 0, f"V = {V}: device error {a.last_error()}"
        assert first_sizes[-1] == final_size, "the total does not depend on V"
        prev, ph = 0, []
        for i in range(4):
            ins = statistics.median(tm.ms(f"ins{i}"))
            rw = statistics.median(tm.ms(f"rw{i}"))
            added = first_sizes[i] - prev
            prev = first_sizes[i]
            ph.append({"insert_us": 1e3 * ins, "insert_Gelem_s": added / (ins * 1e-3) / 1e9,
                       "rw_us": 1e3 * rw, "rw_GBps": 16 * first_sizes[i] / (rw * 1e-3) / 1e9})
        rows.append({"V": V, "tiles_per_lfvector": (n // V + 1023) // 1024, "phases": ph})
        a.close()
        pool.close()
    return rows


def cpu_baseline(rounds, V, min_seconds=10.0, max_reps=4):
    """The CPU oracle (list form, one thread) on the full workload, repeated until
    about min_seconds of work; returns (Gelem/s, seconds per pass, last flatten)."""
    import oracle
    times, flat = [], None
    while len(times) < max_reps and (sum(times) < min_seconds or len(times) < 2):
        o = oracle.Oracle(ELEM, V, F, forms=oracle.FORM_LIST)
        t0 = time.perf_counter()
        for r, n in enumerate(rounds):
            o.insert_gen(oracle.GEN_ROUND_TAG, n, round=r, tag_shift=TAG_SHIFT)
            o.shrink(1, 10)
        o.rw(oracle.OP_MUL3ADD1)
        flat = o.flatten()
        times.append(time.perf_counter() - t0)
        o.close()
    t = statistics.median(times)
    return (1 << 28) / t / 1e9, t, len(times), flat


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.batched_counters:
        batched_counters()
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; only the single-GPU "
                          "path is implemented", "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2209_00103_amd import ggarray as G
    from paper_2209_00103_amd import workloads as wl

    torch.cuda.set_device(0)
    stage("configuration 2")
    V = args.vectors
    rounds = wl.cfg2_round_threads()
    gens = [G.make_gen(G.GEN_ROUND_TAG, round=r, tag_shift=TAG_SHIFT) for r in range(len(rounds))]
    pool = G.Pool(8 << 30)
    arr = G.GGArray(pool, ELEM, V, F)
    prefix_buf = torch.empty(V + 1, dtype=torch.int64, device="cuda")

    # Size the flatten buffer with one untimed pass; capacity / live after each round.
    mem_rounds = []
    for r, n in enumerate(rounds):
        arr.insert_gen(gens[r], n)
        arr.shrink(1, 10)
        live, cap = arr.size(), arr.capacity()
        mem_rounds.append({"round": r, "live": live, "capacity": cap, "capacity_over_live": round(cap / live, 4)})
    final_size = arr.size()
    capacity = arr.capacity()
    pool_stats = pool.stats()
    footprint = arr.footprint()
    arr.shrink(1, 1)
    out = torch.empty(final_size, dtype=torch.int32, device="cuda")
    log(f"final size {final_size}, capacity {capacity} ({capacity / final_size:.3f} x live)")

    for _ in range(args.warmup):
        ggarray_step(G, arr, gens, rounds, out, prefix_buf)
    torch.cuda.synchronize()

    # Timed region: K steps back to back, events only at the two ends.
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        ggarray_step(G, arr, gens, rounds, out, prefix_buf)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    assert arr.last_error() == 0, "device error during the timed steps"
    ms_step = ev0.elapsed_time(ev1) / args.steps
    ms_step_wall = wall * 1e3 / args.steps

    # The same step captured once as a HIP graph and replayed K times (one
    # submission per step instead of about six launches).
    graph_ms = None
    try:
        gs = torch.cuda.Stream()
        gs.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(gs):
            ggarray_step(G, arr, gens, rounds, out, prefix_buf)  # eager on the capture stream first
        gs.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=gs):
            ggarray_step(G, arr, gens, rounds, out, prefix_buf)
        for _ in range(max(1, args.warmup)):
            graph.replay()
        torch.cuda.synchronize()
        g0 = torch.cuda.Event(enable_timing=True)
        g1 = torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(gs):
            g0.record()
            for _ in range(args.steps):
                graph.replay()
            g1.record()
        torch.cuda.synchronize()
        assert arr.last_error() == 0, "device error during the graph replays"
        graph_ms = g0.elapsed_time(g1) / args.steps
        del graph
    except Exception as e:  # reported, never silently dropped
        log(f"graph replay failed: {e!r}\n{traceback.format_exc()}")
    log(f"graph replay: {graph_ms} ms/step")

    arr.shrink(1, 1)  # the fused steps leave the array full; the per-kernel pass starts empty
    torch.cuda.synchronize()

    # Per-kernel durations: the same K steps again with events around every call, and
    # the r/w and flatten kernels timed by events their own dispatches record at the
    # kernel's start and end (the spans around those calls also hold the tile-table
    # launch and the dispatch).
    timer = Timer(torch)
    arr.kernel_timing(True)
    k_rw, k_fl = [], []
    k_ins = [[] for _ in rounds]
    for _ in range(args.steps):
        ggarray_step(G, arr, gens, rounds, out, prefix_buf, timer, k_ins)
        k_rw.append(arr.kernel_ms(0))
        k_fl.append(arr.kernel_ms(1))
    torch.cuda.synchronize()
    assert arr.last_error() == 0, "device error during the per-kernel pass"

    # The clear and the twelve rounds as the timed steps run them, one
    # ggarray_insert_gen_rounds launch (clear_first), timed alone; each rep clears
    # the full array the one before left.
    k_one = []
    arr.insert_gen_rounds(gens, rounds, 1, 10)
    for _ in range(args.steps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        arr.insert_gen_rounds(gens, rounds, 1, 10, clear_first=True)
        e1.record()
        torch.cuda.synchronize()
        k_one.append(e0.elapsed_time(e1))
    arr.shrink(1, 1)
    assert arr.last_error() == 0, "device error during the one-launch rounds"

    # The same r/w and flatten with the caches cold: before each, 1 GiB of unrelated
    # data is read (clean lines), evicting the array from L2 and the 256 MB Infinity
    # Cache, so no byte of it is served from there.
    scratch = torch.ones(1 << 28, dtype=torch.int32, device="cuda")
    k_rw_cold, k_fl_cold = [], []
    for _ in range(args.steps):
        arr.shrink(1, 1)
        for r, n in enumerate(rounds):
            arr.insert_gen(gens[r], n)
            arr.shrink(1, 10)
        arr.prefix_into(prefix_buf)
        scratch.sum()
        arr.rw(G.MUL3ADD1)
        k_rw_cold.append(arr.kernel_ms(0))
        scratch.sum()
        arr.flatten_into(out)
        k_fl_cold.append(arr.kernel_ms(1))
    torch.cuda.synchronize()
    arr.kernel_timing(False)
    del scratch
    assert arr.last_error() == 0, "device error during the cold-cache pass"

    # Access by global index (rw_g, Sec. VI-B) on the final state: r/w x = 3x + 1 by
    # global index beside the bucket-walk r/w, and a gather of 2^24 uniform indices.
    for r, n in enumerate(rounds):
        arr.insert_gen(gens[r], n)
        arr.shrink(1, 10)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(1)
    n_gather = 1 << 24
    gidx = torch.randint(0, final_size, (n_gather,), device="cuda", dtype=torch.int64, generator=gen)
    gout = torch.empty(n_gather, dtype=torch.int32, device="cuda")
    arr.rw_global(G.MUL3ADD1)
    arr.gather(gidx, gout)
    for _ in range(args.steps):
        with timer.span("rw_global"):
            arr.rw_global(G.MUL3ADD1)
        with timer.span("gather"):
            arr.gather(gidx, gout)
    torch.cuda.synchronize()
    assert arr.last_error() == 0, "device error during the global-index pass"
    arr.shrink(1, 1)

    # Per-kernel figures: algorithmic bytes per launch over the measured duration.
    ins_ms = [statistics.mean(k) for k in k_ins]
    ins_span_ms = [statistics.mean(timer.ms(f"insert{r}")) for r in range(len(rounds))]
    rw_ms = statistics.mean(k_rw)
    fl_ms = statistics.mean(k_fl)
    pre_ms = statistics.mean(timer.ms("prefix"))
    clr_ms = statistics.mean(timer.ms("clear"))
    ins_bytes = [ELEM * n for n in rounds]
    rw_bytes = 2 * ELEM * final_size
    fl_bytes = 2 * ELEM * final_size + 8 * (V + 1)
    gbps = lambda b, ms: b / (ms * 1e-3) / 1e9  # noqa: E731
    kernels = {
        "insert": {"launches_per_step": len(rounds), "avg_us": 1e3 * sum(ins_ms) / len(rounds),
                   "bytes_per_launch": sum(ins_bytes) / len(rounds),
                   "GBps": gbps(sum(ins_bytes), sum(ins_ms)),
                   "Gelem_s": (1 << 28) / (sum(ins_ms) * 1e-3) / 1e9,
                   "per_round_us": [round(1e3 * x, 2) for x in ins_ms],
                   "per_round_GBps": [round(gbps(b, ms)) for b, ms in zip(ins_bytes, ins_ms)],
                   # rounds writing less than the 256 MiB Infinity Cache may be served by it
                   "cache_assisted_rounds": [r for r, b in enumerate(ins_bytes) if b < (256 << 20)],
                   "last_round_GBps": gbps(ins_bytes[-1], ins_ms[-1]),
                   "fused": "each launch also applies its round's shrink 1/10 (pops and bucket releases)",
                   "one_launch": {"avg_us": round(1e3 * statistics.mean(k_one), 2),
                                  "Gelem_s": (1 << 28) / (statistics.mean(k_one) * 1e-3) / 1e9,
                                  "GBps": gbps(sum(ins_bytes), statistics.mean(k_one)),
                                  "note": "the clear of the full array, then all twelve rounds and shrinks, "
                                          "in one ggarray_insert_gen_rounds launch, as the timed steps run "
                                          "them; events around the call"},
                   "span_us": round(1e3 * sum(ins_span_ms) / len(rounds), 2),
                   "timing": "events recorded by each launch's own dispatch; span_us: events around the call"},
        "rw": {"launches_per_step": 1, "avg_us": 1e3 * rw_ms, "bytes_per_launch": rw_bytes,
               "GBps": gbps(rw_bytes, rw_ms),
               "cold_cache_GBps": gbps(rw_bytes, statistics.mean(k_rw_cold)),
               "span_us": 1e3 * statistics.mean(timer.ms("rw")),
               "timing": "events recorded by the kernel's own dispatch; span_us: events around the call "
                         "(tile-table launch and dispatch included)"},
        "flatten": {"launches_per_step": 1, "avg_us": 1e3 * fl_ms, "bytes_per_launch": fl_bytes,
                    "GBps": gbps(fl_bytes, fl_ms),
                    "cold_cache_GBps": gbps(fl_bytes, statistics.mean(k_fl_cold)),
                    "span_us": 1e3 * statistics.mean(timer.ms("flatten"))},
        "shrink": {"launches_per_step": 1, "avg_us": 1e3 * clr_ms,
                   "note": "the clear (shrink 1/1); the rounds' shrinks run inside their insertion launches"},
        "prefix_scan": {"launches_per_step": 1, "avg_us": 1e3 * pre_ms},
    }
    rwg_ms = statistics.mean(timer.ms("rw_global"))
    gat_ms = statistics.mean(timer.ms("gather"))
    next_rows = {
        "rw_global": {"avg_us": 1e3 * rwg_ms, "bytes_per_launch": rw_bytes, "GBps": gbps(rw_bytes, rwg_ms),
                      "vs_rw": rw_ms / rwg_ms},
        "gather": {"indices": n_gather, "avg_us": 1e3 * gat_ms, "Gelem_s": n_gather / (gat_ms * 1e-3) / 1e9,
                   "bytes_per_launch": 16 * n_gather, "GBps": gbps(16 * n_gather, gat_ms),
                   "note": "per index: 8 B index + 4 B element + 4 B output; the element read is random"},
    }
    for k, ts in (("insert_all_rounds", [sum(x) for x in zip(*k_ins)]),
                  ("rw", k_rw), ("flatten", k_fl)):
        q = sorted(ts)
        (kernels["insert"] if k == "insert_all_rounds" else kernels[k])["p10_p50_p90_us"] = [
            round(1e3 * q[int(0.1 * (len(q) - 1))], 2), round(1e3 * statistics.median(q), 2),
            round(1e3 * q[int(round(0.9 * (len(q) - 1)))], 2)]
    for k in ("insert", "rw", "flatten"):
        kernels[k]["frac"] = kernels[k]["GBps"] / HBM_PEAK_GBPS
    totals = {"insert": sum(ins_ms), "rw": rw_ms, "flatten": fl_ms}
    dom = max(totals, key=totals.get)
    traffic = measured_traffic(args.traffic, dom)
    roofline = {"kernel": dom, "bound": "hbm", "achieved": kernels[dom]["GBps"], "peak": HBM_PEAK_GBPS,
                "unit": "GB/s", "frac": kernels[dom]["GBps"] / HBM_PEAK_GBPS, "traffic": traffic,
                "avg_launch_us": kernels[dom]["avg_us"], "bytes_per_launch": kernels[dom]["bytes_per_launch"]}
    log(f"ms/step {ms_step:.3f} (wall {ms_step_wall:.3f}); insert {kernels['insert']['Gelem_s']:.1f} Gelem/s "
        f"rw {kernels['rw']['GBps']:.0f} GB/s flatten {kernels['flatten']['GBps']:.0f} GB/s "
        f"(cold caches: rw {kernels['rw']['cold_cache_GBps']:.0f}, flatten {kernels['flatten']['cold_cache_GBps']:.0f})")

    ceilings = None
    if not args.no_ceiling:
        stage("plain-kernel ceilings")
        ceilings = ceiling_leg(torch, final_size)
        ceilings["flatten_over_copy"] = kernels["flatten"]["GBps"] / ceilings["copy"]["GBps"]
        ceilings["rw_over_inplace_add"] = kernels["rw"]["GBps"] / ceilings["inplace_add"]["GBps"]
        same = ceilings["same_size"]
        same["flatten_over_copy"] = kernels["flatten"]["GBps"] / same["copy"]["GBps"]
        same["rw_over_inplace_add"] = kernels["rw"]["GBps"] / same["inplace_add"]["GBps"]
        log(f"plain kernels: fill {ceilings['fill']['GBps']:.0f} GB/s, copy {ceilings['copy']['GBps']:.0f} GB/s, "
            f"in-place add {ceilings['inplace_add']['GBps']:.0f} GB/s; flatten / copy "
            f"{ceilings['flatten_over_copy']:.2f}, rw / in-place add {ceilings['rw_over_inplace_add']:.2f}; "
            f"at the array's size: copy {same['copy']['GBps']:.0f}, in-place add {same['inplace_add']['GBps']:.0f} GB/s "
            f"(flatten / copy {same['flatten_over_copy']:.2f}, rw / in-place add {same['rw_over_inplace_add']:.2f})")

    # Baselines beside it: the static array (pre-allocated for 2^28) and the
    # host-resized array, same insertion rounds (they have no shrink) and r/w.
    baselines = None
    if not args.no_baselines:
        stage("baselines")
        baselines = {}
        st = G.StaticArray(1 << 28, ELEM)
        for rep in range(args.warmup + args.steps):
            st.clear()
            tm = Timer(torch)
            for r, n in enumerate(rounds):
                with tm.span("ins"):
                    st.insert_gen(gens[r], n)
            with tm.span("rw"):
                st.rw(G.MUL3ADD1)
            if rep == args.warmup:
                torch.cuda.synchronize()
                s_ins, s_rw = [], []
            if rep >= args.warmup:
                torch.cuda.synchronize()
                s_ins.append(sum(tm.ms("ins")))
                s_rw.append(tm.ms("rw")[0])
        st_size = st.size()
        assert st.last_error() == 0 and st_size == 1 << 28
        baselines["static"] = {"insert_Gelem_s": (1 << 28) / (statistics.mean(s_ins) * 1e-3) / 1e9,
                               "rw_GBps": gbps(2 * ELEM * st_size, statistics.mean(s_rw)),
                               "capacity_elems": 1 << 28, "live_elems": st_size}
        st.close()
        sem_ins, sem_rw, resizes = [], [], 0
        for rep in range(max(2, min(args.steps, 3)) + 1):
            ss = G.SemiStaticArray(ELEM, rounds[0])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for r, n in enumerate(rounds):
                ss.insert_gen(gens[r], n)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            ss.rw(G.MUL3ADD1)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            if rep > 0:
                sem_ins.append(t1 - t0)
                sem_rw.append(t2 - t1)
            resizes = ss.resizes()
            ss.close()
        baselines["semi_static"] = {"insert_Gelem_s": (1 << 28) / statistics.mean(sem_ins) / 1e9,
                                    "rw_GBps": 2 * ELEM * (1 << 28) / statistics.mean(sem_rw) / 1e9,
                                    "resizes": resizes, "timing": "host wall clock (resizes synchronise)"}
        try:
            baselines["mapped"] = mapped_baseline(G, torch, gens, rounds, args.steps)
        except Exception as e:  # reported, never silently dropped
            baselines["mapped"] = {"error": str(e)}
            log(f"mapped baseline failed: {e!r}\n{traceback.format_exc()}")
        log(f"static insert {baselines['static']['insert_Gelem_s']:.1f} Gelem/s rw "
            f"{baselines['static']['rw_GBps']:.0f} GB/s; semi-static insert "
            f"{baselines['semi_static']['insert_Gelem_s']:.1f} Gelem/s; mapped "
            f"{baselines['mapped'].get('insert_Gelem_s', baselines['mapped'].get('error'))}")

    sparse = None
    if not args.no_baselines:
        stage("sparse rounds")
        try:
            sparse = sparse_leg(G, torch, rounds, V, args.steps, args.warmup)
            log(f"sparse rounds: ggarray {sparse['ggarray']['Gelem_s']:.1f} Gelem/s (last round "
                f"{sparse['ggarray']['last_round_GBps']:.0f} GB/s), static {sparse['static']['Gelem_s']:.1f} "
                f"Gelem/s (last round {sparse['static']['last_round_GBps']:.0f} GB/s); buffer mode last round "
                f"{sparse['ggarray_buffer']['last_round_GBps']:.0f} GB/s against static "
                f"{sparse['static_buffer']['last_round_GBps']:.0f} GB/s")
        except Exception as e:  # reported, never silently dropped
            sparse = {"error": str(e)}
            log(f"sparse leg failed: {e!r}\n{traceback.format_exc()}")

    footprint_end = arr.footprint()  # after the timed steps: the tile table has been built
    arr.close()
    pool.close()
    batched = None
    if not args.no_batched:
        stage("batched")
        batched = batched_leg(G, wl, torch, np, args.steps, args.warmup)
        t = batched["timings"]
        log(f"batched: one launch per phase {t['batched']['mean_ms']:.3f} ms (graph {t['batched_graph']['mean_ms']:.3f}),"
            f" per-array launches {t['per_array']['mean_ms']:.3f} ms (graph {t['per_array_graph']['mean_ms']:.3f});"
            f" one persistent launch {t['persistent']['mean_ms']:.3f} ms (graph {t['persistent_graph']['mean_ms']:.3f});"
            f" identical {batched['batched_equals_per_array']} / {batched['persistent_equals_batched']}")
    shootout = memory_model = None
    if not args.no_shootout:
        stage("shootout, memory model")
        try:
            shootout = shootout_leg(G, torch)
            log("shootout scan/atomic speedup: " + ", ".join(f"2^{20 + i}: {r['scan_speedup']:.2f}"
                                                          for i, r in enumerate(shootout["rows"])))
        except Exception as e:  # reported, never silently dropped
            shootout = {"error": str(e)}
            log(f"shootout failed: {e!r}\n{traceback.format_exc()}")
        try:
            memory_model = memory_model_leg(G, torch, np)
            log("memory model: " + ", ".join(f"s={r['sigma']}: gg {r['ggarray_capacity_over_live']:.2f} "
                                             f"static {r['static_1pct_capacity_over_live']:.2f}"
                                             for r in memory_model["rows"]))
        except Exception as e:
            memory_model = {"error": str(e)}
            log(f"memory model failed: {e!r}\n{traceback.format_exc()}")
    config1 = None
    if not args.no_config1:
        stage("configuration 1")
        try:
            config1 = config1_leg(G, wl, torch)
            o1 = config1["ops"]
            log(f"configuration 1: step {config1['step_us_eager']:.1f} us eager, {config1['step_us_graph']:.1f} us "
                f"as a graph; insert p50 " + ", ".join(f"{o1[f'insert{r}']['p50_us']:.1f}" for r in range(4))
                + f" us, r/w {o1['rw']['p50_us']:.1f} us, flatten {o1['flatten']['p50_us']:.1f} us; persistent step "
                f"{config1['persistent_step']['us_eager']:.1f} us eager, {config1['persistent_step']['us_graph']:.1f} "
                f"us as a graph (identical {config1['persistent_step']['identical']})")
        except Exception as e:  # reported, never silently dropped
            config1 = {"error": str(e)}
            log(f"configuration-1 leg failed: {e!r}\n{traceback.format_exc()}")
    config3 = None
    if not args.no_config3:
        stage("configuration 3")
        try:
            config3 = config3_leg(G, wl, torch)
            r3 = config3["insert_roofline"]
            log("configuration 3: insert " + ", ".join(f"{p['insert_Gelem_s']:.1f}" for p in config3["phases"])
                + f" Gelem/s (VALU issue {r3['frac'] if r3['frac'] is None else round(r3['frac'], 2)} of peak); "
                + "r/w " + ", ".join(f"{p['rw_GBps']:.0f}" for p in config3["phases"])
                + f" GB/s; flatten {config3['flatten_GBps']:.0f} GB/s; buffer mode insert "
                + ", ".join(f"{p['insert_traffic_GBps']:.0f}" for p in config3["buffer_mode"]["phases"])
                + f" GB/s (identical {config3['buffer_mode']['identical_to_gen_mode']})")
        except Exception as e:  # reported, never silently dropped
            config3 = {"error": str(e)}
            log(f"configuration-3 leg failed: {e!r}\n{traceback.format_exc()}")
    two_phase = None
    if not args.no_two_phase:
        stage("two-phase")
        try:
            two_phase = two_phase_leg(G, torch, V)
            log("two-phase speedup flatten+work vs mapped: " + ", ".join(
                f"{key} {r['speedup_flatten_vs_mapped']:.2f}" for key, r in two_phase["rows"].items()))
        except Exception as e:  # reported, never silently dropped
            two_phase = {"error": str(e)}
            log(f"two-phase leg failed: {e!r}\n{traceback.format_exc()}")
    served = None
    if not args.no_served:
        stage("served")
        served = served_leg(G, wl, torch, np, args)
        log(f"served: saturation {served['saturation']['req_per_s']:.3e} req/s; " + "; ".join(
            f"{p['load']}x p50 {p['batched']['all']['p50_us']:.0f} us p99 {p['batched']['all']['p99_us']:.0f} us"
            f" (per-request p99 {p['per_request']['all']['p99_us']:.0f} us)" for p in served["loads"]))

    cpu = None
    parity = None
    if not args.no_cpu:
        stage("cpu oracle")
        rate, secs, reps, ref = cpu_baseline(rounds, V)
        got = G.as_unsigned(out)
        parity = bool(got.shape == ref.shape and np.array_equal(got, ref))
        cpu = {"value": rate, "unit": "Gelem/s", "cores": 1, "kind": "oracle",
               "sample": f"the full workload (2^28 insertions, 12 rounds with shrink, r/w, flatten), "
                         f"single-threaded list-form oracle, median of {reps} passes of {secs:.2f} s",
               "host_cpu": _cpu_model(), "host_nproc": os.cpu_count()}
        log(f"cpu oracle {rate:.4f} Gelem/s ({secs:.2f} s/pass); flatten parity with oracle: {parity}")

    value = (1 << 28) / (ms_step * 1e-3) / 1e9
    line = {
        "metric": METRIC, "value": value, "unit": "Gelem/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "growth at scale: 2^28 uint32 insertions over 12 rounds (live count "
                               "doubling, shrink 1/10 per round), r/w x=3x+1, flatten",
                   "n_vectors": V, "first_bucket": F, "elem": "u32", "inserts": 1 << 28, "rounds": len(rounds),
                   "final_size": final_size},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernels": kernels,
        "baselines": baselines,
        "sparse_rounds": sparse,
        "memory": {"capacity_elems": capacity, "live_elems": final_size, "capacity_over_live": capacity / final_size,
                   "per_round": mem_rounds,
                   "pool_bytes_in_use": pool_stats["in_use"], "pool_high_water": pool_stats["high_water"],
                   "metadata_bytes": footprint["metadata"], "lookback_bytes": footprint["lookback"],
                   "tile_table_bytes": footprint_end["tile_tables"]},
        "ceilings": ceilings,
        "parity_with_oracle": parity,
        "ms_per_step_wall": ms_step_wall,
        "ms_per_step_graph": graph_ms,
        "batched": batched,
        "served": served,
        "global_index_access": next_rows,
        "two_phase": two_phase,
        "config1": config1,
        "config3": config3,
        "insertion_shootout": shootout,
        "memory_model": memory_model,
    }
    # The full record goes to a file; stdout ends with one compact line (a few KB)
    # that carries the headline, the roofline of the dominant kernel and the CPU
    # baseline.
    detail_path = write_detail(line)
    print(json.dumps(headline(line, detail_path)), flush=True)


def write_detail(line) -> str:
    out_dir = os.path.join(ROOT, "gpurun_out")
    os.makedirs(out_dir, exist_ok=True)
    path = os.path.join(out_dir, "bench_detail.json")
    with open(path, "w") as f:
        json.dump(line, f, indent=1)
    return os.path.relpath(path, ROOT)


def _r(x, nd=4):
    return None if x is None else round(float(x), nd)


def headline(line, detail_path):
    """The compact result line: contract keys, roofline, CPU baseline and the
    headline comparisons (insert and r/w against the static array, batched and
    served latency), each a number or null."""
    k = line["kernels"]
    roof = {key: (_r(v) if isinstance(v, float) else v) for key, v in line["roofline"].items()}
    cpu = line["cpu_baseline"]
    if cpu is not None:
        cpu = {"value": _r(cpu["value"], 5), "unit": cpu["unit"], "cores": cpu["cores"], "kind": cpu["kind"],
               "sample": cpu["sample"], "host_cpu": cpu["host_cpu"], "host_nproc": cpu["host_nproc"]}
    head = {"insert_Gelem_s": _r(k["insert"]["Gelem_s"], 1), "rw_GBps": _r(k["rw"]["GBps"], 1),
            "flatten_GBps": _r(k["flatten"]["GBps"], 1), "rw_frac": _r(k["rw"]["frac"]),
            "flatten_frac": _r(k["flatten"]["frac"]), "insert_frac": _r(k["insert"]["frac"]),
            "insert_one_launch_Gelem_s": _r(k["insert"]["one_launch"]["Gelem_s"], 1)}
    bl = line.get("baselines") or {}
    for key, src in (("static", bl.get("static")),):
        if src:
            head[key + "_insert_Gelem_s"] = _r(src.get("insert_Gelem_s"), 1)
            head[key + "_rw_GBps"] = _r(src.get("rw_GBps"), 1)
    sp = line.get("sparse_rounds") or {}
    if "ggarray" in sp:
        head["sparse_insert_Gelem_s"] = _r(sp["ggarray"]["Gelem_s"], 1)
        head["sparse_static_insert_Gelem_s"] = _r(sp["static"]["Gelem_s"], 1)
        head["sparse_last_round_GBps"] = _r(sp["ggarray"]["last_round_GBps"], 1)
        if "ggarray_buffer" in sp:
            head["sparse_buffer_last_round_GBps"] = _r(sp["ggarray_buffer"]["last_round_GBps"], 1)
            head["sparse_buffer_static_last_round_GBps"] = _r(sp["static_buffer"]["last_round_GBps"], 1)
    if bl.get("static"):
        # like for like: both sides timed by events around the calls (dispatch included)
        ins_span = (1 << 28) / (k["insert"]["launches_per_step"] * k["insert"]["span_us"] * 1e-6) / 1e9
        rw_span = k["rw"]["bytes_per_launch"] / (k["rw"]["span_us"] * 1e-6) / 1e9
        head["insert_vs_static"] = _r(ins_span / bl["static"]["insert_Gelem_s"], 3)
        head["rw_vs_static"] = _r(rw_span / bl["static"]["rw_GBps"], 3)
    c3 = line.get("config3") or {}
    if "insert_roofline" in c3:
        head["cfg3_insert_Gelem_s"] = _r(statistics.mean(p["insert_Gelem_s"] for p in c3["phases"]), 1)
        head["cfg3_rw_GBps"] = _r(statistics.mean(p["rw_GBps"] for p in c3["phases"]), 1)
        bm = c3.get("buffer_mode")
        if bm:
            head["cfg3_buffer_insert_GBps"] = _r(bm["insert_roofline"]["achieved"], 1)
            head["cfg3_buffer_insert_frac"] = _r(bm["insert_roofline"]["frac"])
            head["cfg3_buffer_identical"] = bm["identical_to_gen_mode"]
    bt = (line.get("batched") or {}).get("timings")
    if bt:
        head["batched_ms"] = _r(bt["batched"]["mean_ms"], 3)
        head["batched_graph_ms"] = _r(bt["batched_graph"]["mean_ms"], 3)
        head["per_array_ms"] = _r(bt["per_array"]["mean_ms"], 3)
        head["batched_persistent_ms"] = _r(bt["persistent"]["mean_ms"], 3)
        head["batched_persistent_graph_ms"] = _r(bt["persistent_graph"]["mean_ms"], 3)
    sv = line.get("served")
    if sv:
        head["served_saturation_req_s"] = _r(sv["saturation"]["req_per_s"], 0)
        head["served_loads"] = [{"load": p["load"], "p50_us": _r(p["batched"]["all"]["p50_us"], 1),
                                 "p99_us": _r(p["batched"]["all"]["p99_us"], 1)} for p in sv["loads"]]
        m = sv.get("matched") or []
        head["served_matched"] = [{"offered_req_s": _r(p["offered_req_per_s"], 0),
                                   "batched_p50_us": _r(p["batched"]["all"]["p50_us"], 1),
                                   "batched_p99_us": _r(p["batched"]["all"]["p99_us"], 1),
                                   "per_request_p50_us": _r(p["per_request"]["all"]["p50_us"], 1),
                                   "per_request_p99_us": _r(p["per_request"]["all"]["p99_us"], 1)} for p in m]
    c1 = line.get("config1") or {}
    if "step_us_eager" in c1:
        head["cfg1_step_us"] = _r(c1["step_us_eager"], 1)
        head["cfg1_persistent_step_us"] = _r(c1["persistent_step"]["us_eager"], 1)
        head["cfg1_persistent_graph_us"] = _r(c1["persistent_step"]["us_graph"], 1)
    out = {key: line[key] for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
                                      "higher_is_better", "scaling", "vs_baseline", "dtype", "data")}
    out["value"] = _r(out["value"], 3)
    out["ms_per_step"] = _r(out["ms_per_step"], 4)
    out["config"] = line["config"]
    out["roofline"] = roof
    out["cpu_baseline"] = cpu
    out["headline"] = head
    out["parity_with_oracle"] = line["parity_with_oracle"]
    out["ms_per_step_graph"] = _r(line["ms_per_step_graph"], 4)
    out["detail"] = detail_path
    return out


if __name__ == "__main__":
    main()
