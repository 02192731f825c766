#!/usr/bin/env python3
"""Benchmark: RP-Tuning prune sweep (and GreedySearch) on one MI355X.

One step = one pass of the prune hot path over the whole graph: RobustPrune
of every vertex's base out-list at every alpha of the sweep (one launch of
the batched kernel).  Default workload: 1,000,000 uint8 points, d = 128,
64-component Gaussian mixture; base graph = exact 128-NN lists pruned at
alpha = 6/5, R = 64; sweep alpha in {23/20, 11/10, 21/20, 1}, R = 64.

Inputs are resident in HBM before the timed region.  The plain one-workgroup
per-vertex kernel is timed on the same inputs (one launch per alpha), the
search leg reports QPS and recall on the pruned graphs, and the CPU oracle is
timed on a bounded node sample on the host.

Prints ONE JSON line.
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

METRIC = ("RP-Tuning prune nodes/s (+% HBM/MFMA roofline) vs plain FP32; "
          "search QPS, p99 at equal recall")
HBM_PEAK_GBS = 8000.0


COPY_BYTES = 256 << 20
PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SRC = {"u8": os.path.join(ROOT, "paper_2602_08097_amd", "csrc", "k_prune_u8.hip")}


def source_digest(path):
    import hashlib

    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(dtype, n):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary, if it was taken on the current kernel source and workload size."""
    import numpy as np

    path = os.path.join(PROFILES, "prune_u8_sift_u8_traffic.json")
    if dtype != np.uint8 or not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("source_sha256_16") != source_digest(KERNEL_SRC["u8"]) or t.get("n") != n:
        return None
    return t.get("traffic_bytes_per_launch")


def _read_csvs(root, suffix):
    import csv
    import glob

    rows = []
    for path in sorted(glob.glob(os.path.join(root, "**", f"*{suffix}"), recursive=True)):
        with open(path) as f:
            rows.extend(csv.DictReader(f))
    return rows


def _col(row, *names):
    low = {k.lower(): k for k in row}
    for nm in names:
        if nm.lower() in low:
            return row[low[nm.lower()]]
    raise KeyError(f"none of {names} in {list(row)}")


def summarize_profile(root):
    """Summarise the three rocprofv3 runs under root (trace/, fetch/, write/)."""
    out = os.path.join(root, "summary")
    os.makedirs(out, exist_ok=True)
    stats = _read_csvs(os.path.join(root, "trace"), "kernel_stats.csv")
    lines = ["| kernel | calls | average (us) | total (ms) |", "|---|---|---|---|"]
    prune_avg_ns = None
    for r in stats:
        name = _col(r, "Name", "KERNEL_NAME")
        calls = int(_col(r, "Calls"))
        avg = float(_col(r, "AverageNs", "Average_Ns", "AVERAGE_NS"))
        tot = float(_col(r, "TotalDurationNs", "Total_Duration_Ns", "TOTAL_DURATION_NS"))
        if "prune" in name or calls >= 3:
            lines.append(f"| {name[:90]} | {calls} | {avg / 1e3:.1f} | {tot / 1e6:.2f} |")
        if "prune_u8_kernel" in name:
            prune_avg_ns = avg
    res = {"prune_u8_avg_ns": prune_avg_ns}
    for tag in sorted(os.listdir(root)):
        if tag in ("trace", "summary") or not os.path.isdir(os.path.join(root, tag)):
            continue
        rows = _read_csvs(os.path.join(root, tag), "counter_collection.csv")
        per = {}
        for r in rows:
            counter = _col(r, "Counter_Name", "COUNTER_NAME")
            name = _col(r, "Kernel_Name", "KERNEL_NAME")
            disp = _col(r, "Dispatch_Id", "DISPATCH_ID")
            per.setdefault((counter, name), {}).setdefault(disp, 0.0)
            per[(counter, name)][disp] += float(_col(r, "Counter_Value", "COUNTER_VALUE"))
        for (counter, name), d in sorted(per.items()):
            vals = list(d.values())
            res[f"{counter} per dispatch (n={len(vals)}): {name[:100]}"] = sum(vals) / len(vals)
    with open(os.path.join(out, "kernel_stats.md"), "w") as f:
        f.write("\n".join(lines) + "\n")
    with open(os.path.join(out, "counters.json"), "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res, indent=1))


def load_or_build(args, spec, dev):
    import numpy as np

    import workloads

    if args.cache and os.path.exists(args.cache):
        z = np.load(args.cache, allow_pickle=False)
        tg = z["targets"] if z["targets"].size else None
        return workloads.Workload(spec, z["X"], z["Q"], z["knn"], z["knn_deg"], int(z["start"]),
                                  tg, z["sample"])
    w = workloads.build(args.config, n=args.n, nq=args.nq, device=dev)
    if args.cache:
        np.savez(args.cache, X=w.X, Q=w.Q, knn=w.knn, knn_deg=w.knn_deg, start=np.int64(w.start),
                 targets=w.targets if w.targets is not None else np.zeros(0, np.int32),
                 sample=w.sample)
    return w


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes(deg, d, esz, Rs_per_output):
    """Bytes RP-Tuning must move per sweep: per vertex the list (4(m+1)), the
    candidate and own rows ((m+1) d e) and every output row (4R + 4)."""
    import numpy as np

    m = deg.astype(np.int64)
    per_out = sum(4 * R + 4 for R in Rs_per_output)
    return int((4 * (m + 1) + (m + 1) * d * esz).sum() + per_out * m.shape[0])


MFMA_PEAK = {"u8": 5000.0, "f32": 2500.0}  # dense int8 TOP/s, fp16 TFLOP/s


def mfma_usage(dtype, deg, d, r_max, kernel_ms):
    """Matrix-unit work of one sweep launch: the executed MFMA operations of
    the batched kernel (uint8: six 32 x 32 x 32 int8 products per vertex and
    32-dimension step, three Gram blocks and three with x_p in every row, over
    4 steps for d <= 128 and 8 above; float32: the blocks on and above the diagonal of the
    row blocks in use, three 32 x 32 x 16 FP16 products per 16-dimension step)
    and the Gram's useful work (one product per candidate pair above the
    diagonal), each over the kernel's mean time, against the dense peak."""
    import numpy as np

    m = deg.astype(np.int64)
    if dtype == np.uint8:
        steps = 4 if d <= 128 else 8
        executed = int(m.shape[0]) * 6 * steps * (32 * 32 * 32 * 2)
        key, unit = "u8", "TOP/s"
    else:
        nbu = np.maximum(1, np.minimum((r_max + 31) // 32, (m + 31) // 32))
        steps = (d + 15) // 16
        executed = int((nbu * (nbu + 1) // 2).sum()) * 3 * steps * (32 * 32 * 16 * 2)
        key, unit = "f32", "TFLOP/s"
    useful = int((m * (m - 1) // 2).sum()) * d * 2
    sec = kernel_ms * 1e-3
    peak = MFMA_PEAK[key]
    ach = executed / sec / 1e12
    return {"unit": unit, "executed": round(ach, 2), "peak": peak, "frac": round(ach / peak, 4),
            "gram_useful": round(useful / sec / 1e12, 2),
            "executed_ops_per_launch": executed}


def batched_kernel_name(dtype, r_max, d):
    """The kernel the sweep dispatches to for this graph shape."""
    import numpy as np

    if dtype == np.uint8:
        return "prune_u8_kernel" if r_max <= 64 and d % 16 == 0 and d <= 256 else \
            "prune_plain_kernel"
    return "prune_f32_kernel" if r_max <= 96 else "prune_plain_kernel"


def exact_gt_u8(X, Q, k, chunk=1024):
    """Exact top-k by (S, id) for uint8 data on the GPU (integer keys)."""
    import torch

    n = X.shape[0]
    idbits = max(1, int(n - 1).bit_length())
    Xf = X.float()
    nx = (X.long() ** 2).sum(1)
    rows = torch.arange(n, device=X.device, dtype=torch.int64)
    out = []
    for a in range(0, Q.shape[0], chunk):
        q = Q[a:a + chunk]
        ip = (q.float() @ Xf.T).long()
        key = (nx[None, :] - 2 * ip + (q.long() ** 2).sum(1)[:, None]) << idbits | rows[None, :]
        vals, _ = torch.topk(key, k, dim=1, largest=False, sorted=True)
        out.append((vals & ((1 << idbits) - 1)).to(torch.int32))
    return torch.cat(out)


def exact_gt_f32(X, Q, k, chunk=256):
    """Top-k by FP32 squared distance (used for recall only)."""
    import torch

    nx = (X * X).sum(1)
    out = []
    for a in range(0, Q.shape[0], chunk):
        q = Q[a:a + chunk]
        dist = nx[None, :] - 2.0 * (q @ X.T) + (q * q).sum(1)[:, None]
        out.append(torch.topk(dist, k, dim=1, largest=False, sorted=True).indices.to(torch.int32))
    return torch.cat(out)


def reachable_fraction(nbr, deg, start):
    """Fraction of vertices reachable from the start vertex (BFS on the GPU)."""
    import torch

    n, r = nbr.shape
    seen = torch.zeros(n, dtype=torch.bool, device=nbr.device)
    seen[start] = True
    frontier = torch.tensor([start], dtype=torch.int64, device=nbr.device)
    cols = torch.arange(r, device=nbr.device)
    while frontier.numel():
        rows = nbr[frontier]
        nxt = rows[cols[None, :] < deg[frontier][:, None]].long()
        nxt = torch.unique(nxt[~seen[nxt]])
        seen[nxt] = True
        frontier = nxt
    return float(seen.float().mean().item())


def recall(ids, gt, k):
    import torch

    a = ids[:, :k].long()
    b = gt[:, :k].long()
    hit = (a[:, :, None] == b[:, None, :]).any(dim=2).sum().item()
    return hit / (k * a.shape[0])


def cpu_baseline(w, spec, budget_s):
    """The oracle (single thread) on a node sample of the same sweep."""
    import numpy as np

    import oracle
    import workloads

    nodes = workloads.node_sample(w.X.shape[0], 40_000)
    # the oracle builds its own base rows for the sample from the K-NN lists
    b_nbr, b_deg, _ = oracle.prune_graph(w.X, w.knn, w.knn_deg, *spec.base_alpha, spec.base_R,
                                         nodes=nodes)
    n = w.X.shape[0]
    full_nbr = np.zeros((n, spec.base_R), np.int32)
    full_deg = np.zeros(n, np.int32)
    full_nbr[nodes] = b_nbr
    full_deg[nodes] = b_deg
    done = 0
    t0 = time.perf_counter()
    chunk = 500
    while done < len(nodes) and time.perf_counter() - t0 < budget_s:
        part = nodes[done:done + chunk]
        for a in spec.sweep:
            for R in spec.Rs:
                oracle.prune_graph(w.X, full_nbr, full_deg, *a, R, nodes=part)
        done += len(part)
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "nodes/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} sampled vertices x {len(spec.sweep)} alphas x {len(spec.Rs)} R "
                      f"(base rows from the oracle's own RobustPrune of the K-NN lists), "
                      f"{dt:.1f} s single-threaded"}


def serve_trace(spec, n_req, rate, n_graph_ids, Qpool, dev, seed):
    """A Poisson mix: 5% prune requests (alpha ~ U{100..120}/100, R in {32, 48, 64}),
    95% query batches (size floor(exp U[0, ln 4096]), k in {10, 100},
    L in {100, 200, 400}) against the base graph or one of the last six graphs
    requested (what the budget keeps resident)."""
    import math

    import numpy as np
    import torch

    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    made = []
    q0 = 0
    for i in range(n_req):
        t += rng.exponential(1.0 / rate)
        if i == 0 or rng.random() < 0.05:
            a = (int(rng.integers(100, 121)), 100)
            R = int(rng.choice(spec.Rs))
            if (a, R) in made:
                made.remove((a, R))
            made = (made + [(a, R)])[-6:]
            out.append(("prune", t, a, R, None))
        else:
            nq = int(math.floor(math.exp(rng.uniform(0.0, math.log(4096)))))
            if q0 + nq > Qpool.shape[0]:
                q0 = 0
            k = int(rng.choice([10, 100]))
            L = int(rng.choice([100, 200, 400]))
            j = int(rng.integers(0, len(made) + 1))
            a, R = (None, 0) if j == len(made) else made[j]
            out.append(("query", t, a, R, (q0, nq, k, L)))
            q0 += nq
    return out


def serve_run(server, trace, Qpool, dev):
    import numpy as np
    import torch

    reqs, arr, kinds, nqs = [], [], [], []
    for i, (kind, t, a, R, q) in enumerate(trace):
        if kind == "prune":
            reqs.append(server.prune_request(a, R, tag=i))
            nqs.append(0)
        else:
            q0, nq, k, L = q
            ids = torch.empty((nq, k), dtype=torch.int32, device=dev)
            reqs.append(server.query_request(a, R, Qpool[q0:q0 + nq], k, L, ids, tag=i))
            nqs.append(nq)
        arr.append(t)
        kinds.append(kind)
    comps = server.replay(reqs, arr)
    stats = server.stats()
    lat = np.array([c.t_done - c.t_submit for c in comps])
    bad = sum(1 for c in comps if c.status != 0)
    t0 = min(c.t_submit for c in comps)
    t1 = max(c.t_done for c in comps)
    kinds = np.array(kinds)
    nqs = np.array(nqs)
    res = {"makespan_s": t1 - t0, "errors": bad, "stats": stats}
    for kind in ("prune", "query"):
        sel = kinds == kind
        if sel.any():
            res[kind] = {"count": int(sel.sum()),
                         "p50_ms": float(np.percentile(lat[sel], 50) * 1e3),
                         "p99_ms": float(np.percentile(lat[sel], 99) * 1e3),
                         "mean_ms": float(lat[sel].mean() * 1e3)}
    res["qps"] = float(nqs.sum() / (t1 - t0))
    res["queries"] = int(nqs.sum())
    return res


def serve_main(args):
    """Serving benchmark on the 10M x 128 uint8 workload (or --n)."""
    import numpy as np
    import torch

    import workloads
    from paper_2602_08097_amd import Graph, Server

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    spec = workloads.CONFIGS["serve_u8"]
    t0 = time.time()
    w = workloads.build("serve_u8", n=args.n, nq=args.nq, device=dev)
    n, d = w.X.shape
    log(f"serve workload: n={n} d={d} ({time.time() - t0:.1f} s incl. component 128-NN)")
    X = torch.from_numpy(w.X).to(dev)
    g_knn = Graph(X, torch.from_numpy(w.knn).to(dev), torch.from_numpy(w.knn_deg).to(dev), w.start)
    t0 = time.time()
    nb, dg = g_knn.prune(spec.base_alpha, spec.base_R)
    torch.cuda.synchronize()
    log(f"base graph alpha={spec.base_alpha} R={spec.base_R}: {time.time() - t0:.1f} s")
    g_knn.free()
    start = w.start
    del w
    base = Graph(X, nb, dg, start)
    Qpool = torch.from_numpy(workloads.make_queries(spec, spec.nq)).to(dev)
    budget = 6 * n * 65 * 4 + (1 << 20)
    # the plain kernel's time for one prune request at this size
    pn, pd = base.prune_plain((110, 100), 64)
    torch.cuda.synchronize()
    tp = time.perf_counter()
    base.prune_plain((110, 100), 64, out=(pn, pd))
    torch.cuda.synchronize()
    plain_ms = (time.perf_counter() - tp) * 1e3
    tb = time.perf_counter()
    base.prune((110, 100), 64, out=(pn, pd))
    torch.cuda.synchronize()
    one_ms = (time.perf_counter() - tb) * 1e3
    del pn, pd
    log(f"one prune request: plain kernel {plain_ms:.1f} ms, batched kernel {one_ms:.1f} ms")
    rates = [float(r) for r in args.rates.split(",")]
    runs = []
    for rate in rates:
        trace = serve_trace(spec, args.requests, rate, 0, Qpool, dev, seed=int(rate))
        row = {"rate_req_s": rate}
        for mode, fifo in (("batched", 0), ("fifo", 1)):
            server = Server(base, budget, n_streams=4, max_query_batch=8192, fifo=fifo)
            r = serve_run(server, trace, Qpool, dev)
            server.close()
            torch.cuda.synchronize()
            row[mode] = r
            log(f"rate {rate:g}/s {mode}: query p50 {r['query']['p50_ms']:.2f} ms "
                f"p99 {r['query']['p99_ms']:.2f} ms, prune p50 {r.get('prune', {}).get('p50_ms', 0):.1f} ms "
                f"p99 {r.get('prune', {}).get('p99_ms', 0):.1f} ms, {r['qps']:.3e} QPS, "
                f"makespan {r['makespan_s']:.2f} s, sweeps {r['stats']['sweeps']} "
                f"({r['stats']['swept_alphas']} alphas), searches {r['stats']['searches']}, "
                f"evictions {r['stats']['evictions']}")
        runs.append(row)
    top = runs[-1]["batched"]
    line = {"metric": "serving: query and prune request latency p50/p99 with throughput",
            "value": top["qps"], "unit": "queries/s", "n_gpus": 1,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
            "data": "synthetic",
            "config": {"workload": f"serve_u8: {n} x {d} uint8 mixture, base RobustPrune 6/5 "
                                   f"R=64 over component-restricted 128-NN; Poisson mix "
                                   f"5% prune / 95% query batches, {args.requests} requests "
                                   f"per rate", "budget_bytes": budget,
                       "plain_prune_ms": plain_ms, "batched_one_prune_ms": one_ms},
            "runs": runs}
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="sift_u8")
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--nq", type=int, default=None)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-search", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--profile", action="store_true",
                    help="profiling run: a 256 MiB device copy for counter calibration, then "
                         "the timed sweep only (no plain/search/CPU legs)")
    ap.add_argument("--cache", metavar="NPZ",
                    help="load the generated workload from NPZ if present, else generate and save "
                         "it there (for repeated profiler runs)")
    ap.add_argument("--serve", action="store_true",
                    help="serving benchmark: Poisson mix of prune requests and query batches "
                         "through the request loop vs the one-at-a-time FIFO baseline")
    ap.add_argument("--rates", default="100,200,400",
                    help="serving: request arrival rates (requests/s)")
    ap.add_argument("--requests", type=int, default=2000, help="serving: requests per rate")
    ap.add_argument("--summarize-profile", metavar="DIR",
                    help="summarise rocprofv3 output under DIR (trace, fetch, write runs) into "
                         "DIR/summary and exit")
    args = ap.parse_args()

    if args.summarize_profile:
        summarize_profile(args.summarize_profile)
        return
    if args.serve:
        if args.gpus != 1:
            print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
            sys.exit(2)
        serve_main(args)
        return
    if args.profile:
        args.no_plain = args.no_search = args.no_cpu = True

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                                   "(multi-GPU sharding is described in DESIGN.md, not built)"}))
        sys.exit(2)

    import numpy as np
    import torch

    import workloads
    from paper_2602_08097_amd import Graph

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.profile:
        # counter calibration: a plain device copy of a known size
        # (a fill kernel writes COPY_BYTES; a reduction reads COPY_BYTES)
        src = torch.randint(0, 255, (COPY_BYTES,), dtype=torch.uint8, device=dev)
        for _ in range(3):
            total = src.sum(dtype=torch.int64)
        torch.cuda.synchronize()
        del src, total
    spec = workloads.CONFIGS[args.config]
    t0 = time.time()
    w = load_or_build(args, spec, dev)
    n, d = w.X.shape
    log(f"workload {spec.name}: n={n} d={d} ({time.time() - t0:.1f} s incl. exact {spec.knn_k}-NN)")

    X = torch.from_numpy(w.X).to(dev)
    knn = torch.from_numpy(w.knn).to(dev)
    kdeg = torch.from_numpy(w.knn_deg).to(dev)
    g_knn = Graph(X, knn, kdeg, w.start)
    base_nbr, base_deg = g_knn.prune(spec.base_alpha, spec.base_R)
    if w.targets is not None:
        # uneven out-degrees: keep the first min(t_p, deg) ids of each base list
        base_deg = torch.minimum(base_deg, torch.from_numpy(w.targets).to(dev))
        cols = torch.arange(spec.base_R, device=dev, dtype=torch.int32)
        base_nbr = torch.where(cols[None, :] < base_deg[:, None], base_nbr,
                               torch.full_like(base_nbr, -1))
    torch.cuda.synchronize()
    g = g_knn.derive(base_nbr, base_deg)
    deg_np = base_deg.cpu().numpy()
    log(f"base graph alpha={spec.base_alpha} R={spec.base_R}: mean degree {deg_np.mean():.2f}")

    nr = len(spec.Rs)
    outs = [g._outs(spec.Rs[o % nr]) for o in range(len(spec.sweep) * nr)]
    stream = torch.cuda.current_stream()

    # ---- launch tuning (vertices per workgroup), then the timed sweep -------
    tune = g.autotune_sweep(spec.sweep, spec.Rs, outs=outs)
    log(f"autotune: {tune['waves']} vertices per workgroup (ms for 1/2/4/8: "
        f"{[round(x, 3) for x in tune['ms']]})")
    for _ in range(args.warmup):
        g.prune_sweep(spec.sweep, spec.Rs, outs=outs)
    torch.cuda.synchronize()
    g.counters(reset=True)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    t_start = time.perf_counter()
    for e0, e1 in evs:
        e0.record(stream)
        g.prune_sweep(spec.sweep, spec.Rs, outs=outs)
        e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    kern_ms = [e0.elapsed_time(e1) for e0, e1 in evs]
    ctr = g.counters()
    ms_per_step = wall * 1e3 / args.steps
    value = n / (wall / args.steps)
    avg_kernel_ms = float(np.mean(kern_ms))
    out_degs = [o[1].cpu().numpy() for o in outs]
    log(f"batched sweep: {ms_per_step:.3f} ms/step, kernel {avg_kernel_ms:.3f} ms avg, "
        f"{value:.3e} nodes/s; mean out-degree per alpha "
        f"{[round(float(x.mean()), 2) for x in out_degs]}")

    gram_err = None
    if w.X.dtype == np.float32 and spec.base_R <= 96:
        smp = torch.from_numpy(w.sample[:2000].astype(np.int32)).to(dev)
        gram_err = g.gram_error(smp)
        log(f"distance error of the FP16 Gram vs canonical FP64 on 2000 vertices: "
            f"max rel {gram_err['max_rel']:.3e}, mean rel {gram_err['mean_rel']:.3e}, "
            f"max error / proven band {gram_err['max_err_over_bound']:.3f} "
            f"({gram_err['pairs']} pairs)")

    esz = 1 if w.X.dtype == np.uint8 else 4
    Rs_out = [spec.Rs[o % nr] for o in range(len(spec.sweep) * nr)]
    abytes = algorithmic_bytes(deg_np, d, esz, Rs_out)
    achieved = abytes / (avg_kernel_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(w.X.dtype, n),
                "kernel": batched_kernel_name(w.X.dtype, spec.base_R, d),
                "algorithmic_bytes_per_launch": abytes,
                "kernel_ms_avg": round(avg_kernel_ms, 4)}
    mfma = mfma_usage(w.X.dtype, deg_np, d, spec.base_R, avg_kernel_ms)
    log(f"matrix units: {mfma['executed']} {mfma['unit']} executed "
        f"({100 * mfma['frac']:.1f}% of peak), Gram useful {mfma['gram_useful']} {mfma['unit']}")

    # ---- plain kernel on the same inputs ----------------------------------
    plain = None
    if not args.no_plain:
        psteps = max(1, min(3, args.steps))
        pouts = [g._outs(R) for R in spec.Rs]
        for a in spec.sweep:  # warm
            for ir, R in enumerate(spec.Rs):
                g.prune_plain(a, R, out=pouts[ir])
        torch.cuda.synchronize()
        tp = time.perf_counter()
        for _ in range(psteps):
            for a in spec.sweep:
                for ir, R in enumerate(spec.Rs):
                    g.prune_plain(a, R, out=pouts[ir])
        torch.cuda.synchronize()
        pwall = (time.perf_counter() - tp) / psteps
        # the plain path agrees with the batched one (last alpha compared)
        same = bool(torch.equal(pouts[-1][0], outs[-1][0]))
        plain = {"nodes_per_s": n / pwall, "ms_per_step": pwall * 1e3,
                 "speedup_batched_vs_plain": (n / (wall / args.steps)) / (n / pwall),
                 "outputs_identical": same}
        log(f"plain: {pwall * 1e3:.3f} ms/step, {n / pwall:.3e} nodes/s, identical={same}")

    # ---- search leg --------------------------------------------------------
    search = None
    if not args.no_search and w.Q.shape[0] > 0:
        Q = torch.from_numpy(w.Q).to(dev)
        k = spec.k
        gt = exact_gt_u8(X, Q, k) if w.X.dtype == np.uint8 else exact_gt_f32(X, Q, k)
        res = []
        graphs = [("base", g, None)]
        for o in range(0, len(outs), nr):
            graphs.append((f"alpha={spec.sweep[o // nr][0]}/{spec.sweep[o // nr][1]}",
                           g.derive(outs[o][0], outs[o][1]), None))
        reach = {}
        for name, gg, _ in graphs:
            nb_, dg_ = (base_nbr, base_deg) if name == "base" else outs[
                nr * [x[0] for x in graphs[1:]].index(name)]
            reach[name] = reachable_fraction(nb_, dg_, w.start)
            log(f"graph {name}: {100 * reach[name]:.2f}% of vertices reachable from the start")
            for L in spec.Ls:
                gg.search(Q, k, L, want_dist=False)
                torch.cuda.synchronize()
                lat = []
                for _ in range(3):
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                    ids, _, hops = gg.search(Q, k, L, want_dist=False)
                    e1.record(stream)
                    torch.cuda.synchronize()
                    lat.append(e0.elapsed_time(e1))
                ms = float(np.median(lat))
                rec = recall(ids, gt, k) if gt is not None else None
                res.append({"graph": name, "L": L, "qps": Q.shape[0] / (ms * 1e-3),
                            "batch_ms_p50": ms, "batch_ms_max": float(np.max(lat)),
                            "recall_at_k": rec, "mean_hops": float(hops.float().mean().item())})
                log(f"search {name} L={L}: {Q.shape[0] / (ms * 1e-3):.3e} QPS, recall {rec}")
        search = {"k": k, "nq": int(Q.shape[0]), "reachable_fraction": reach, "results": res}

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(w, spec, args.cpu_budget)
        log(f"cpu oracle: {cpu['value']:.1f} nodes/s ({cpu['sample']})")

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "nodes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8" if w.X.dtype == np.uint8 else "f32",
        "data": "synthetic",
        "config": {"workload": f"{spec.name}: {n} x {d} "
                               f"{'uint8' if esz == 1 else 'float32'} Gaussian mixture, base "
                               f"exact {spec.knn_k}-NN + RobustPrune alpha={spec.base_alpha[0]}/"
                               f"{spec.base_alpha[1]} R={spec.base_R}; sweep alpha="
                               f"{[f'{a}/{b}' for a, b in spec.sweep]} R={list(spec.Rs)}",
                   "n": n, "d": d, "mean_base_degree": float(deg_np.mean()),
                   "rechecks_per_node_alpha": ctr["rechecks"] / max(1, ctr["nodes"]),
                   "vertices_per_workgroup": tune["waves"],
                   "outputs_per_step": len(outs)},
        "roofline": roofline,
        "mfma": mfma,
        "distance_error": gram_err if gram_err is not None else
        ({"max_rel": 0.0, "mean_rel": 0.0, "note": "uint8: exact int32 distances"}
         if w.X.dtype == np.uint8 else None),
        "cpu_baseline": cpu,
        "plain": plain,
        "search": search,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
