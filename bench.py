"""Benchmark: triangle count throughput (input edges/s) on one MI355X.

One step = one full pass of the method over the resident graph: BFS levels,
the E0/E1 partition, bucketing and the intersections, ending with the uint64
count on the host (tc_count with no levels given).  The CSR is built on the
GPU beforehand (the paper's input is the CSR) and stays resident in HBM.

Prints one JSON line.  Headline workload: Graph500-style Kronecker graph,
scale 24 (16.8 M vertices, 268 M generated edges), edgefactor 16, initiator
(.57, .19, .19, .05), seed 1, int32 CSR, the degree-threshold heuristic
schedule.  `value` = m / mean step time.

Beside it (in `config`):
  * learned_schedule -- the same steps under the strategy table of the
    stored cost network (paper_2309_09064_amd/sched_net.json), trained on
    whole-pass measurements of other graphs (Kronecker scale 22, seeds 2 and
    3; Chung-Lu 2^20, seed 2) than the ones timed; heuristic and learned
    steps alternate, so drift hits both alike.  `python bench.py
    --train-schedule PATH` measures and trains it anew;
  * secondary -- Chung-Lu 2^22 (power law, gamma 2.1, mean degree 32) under
    both schedules; Kronecker scale 20 with the forward-hashed, per-vertex,
    per-edge and Algorithm 3 / degree-relabel legs; the 4096-graph batch
    (tiles tuned on the union; the eager batched call and the replays of
    its captured plan, all 4096 counts checked against the oracle's).

`roofline` describes the intersection kernel (k_isect) on the headline
graph: its algorithmic bytes B_alg per launch over its mean duration, taken
from HIP events that the library records around the launch on the stream it
launches on, during the timed steps.  `traffic` comes from the committed
counter summary in profiles/ and is null when the kernel sources have
changed since those counters were taken.

`cpu_baseline` is the oracle's sorted-merge edge iterator on the host cores
of this machine, timed on a bounded sample of the headline graph's edges
(interleaved slices of 1/1024 of the CSR entries each, run until about 15 s
of work; its time is scaled by the share of entries sampled); the oracle's
serial BFS + Algorithm 4 counts on the whole scale-20 graph are a second,
stated figure.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "input edges/s + % HBM peak, plain vs learned-scheduled, counts bit-exact"
HBM_PEAK_GBS = 8000.0
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "k_isect_kronecker_s24_traffic.txt")
GOLDEN = os.path.join(ROOT, "tests", "golden", "large_counts.txt")
BATCH_GOLDEN = os.path.join(ROOT, "tests", "golden", "batch_counts.txt")
BATCH_TUNE_SPACE = {"chunk_work": [16384, 32768, 65536], "wave_slots": [1024, 2048], "wg_slots": [16384, 32768],
                    "grid_blocks": [0]}
KERNEL_SOURCES = ("paper_2309_09064_amd/csrc/tc_count.hip", "paper_2309_09064_amd/csrc/tc_internal.hpp")
COPY_PROBE_BYTES = 1 << 30
CPU_SLICE = 1024          # a CPU-baseline slice is every 1024th CSR entry
CPU_SECONDS = 15.0        # slices are run until this much time has passed
TRAIN_GRAPHS = (("kronecker", 22, 2), ("kronecker", 22, 3), ("chunglu", 20, 2))
SCHED_NET = os.path.join(ROOT, "paper_2309_09064_amd", "sched_net.json")
SCHED_MARGIN = 1.0        # predicted gain (sgnlog2 ps per element) a change must exceed
GAIN_NOISE = 0.01         # a learned table counts as faster only beyond this relative gain


def kernel_source_hash():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def b_alg(rp, col, levels):
    """Algorithmic bytes of the intersection pass, from torch tensors (any
    device): every live intersection streams its smaller list once (4 B an
    element), every owner list is read once, plus 8 B per oriented
    horizontal edge and 8 B per vertex (its list records).  Lists: N0+ (the
    rank-oriented horizontal neighbours, rank = (degree, id)) and N1 (the
    neighbours on other levels)."""
    import torch
    n = rp.numel() - 1
    dev = rp.device
    deg = (rp[1:] - rp[:-1]).to(torch.int64)
    u = torch.repeat_interleave(torch.arange(n, device=dev, dtype=torch.int32), deg)
    v = col.to(torch.int32)
    hor = levels[u.long()] == levels[v.long()]
    d0 = torch.bincount(u[hor], minlength=n)
    d1 = deg - d0
    du, dv = deg[u.long()], deg[v.long()]
    up = hor & ((dv > du) | ((dv == du) & (v > u)))
    del du, dv, hor
    d0p = torch.bincount(u[up], minlength=n)
    eu, ev = u[up].long(), v[up].long()
    del u, v
    smin = (torch.minimum(d1[eu], d1[ev]).sum(dtype=torch.int64) +
            torch.minimum(d0p[eu], d0p[ev]).sum(dtype=torch.int64))
    total = 4 * int(smin) + 4 * int(d1.sum() + d0p.sum()) + 8 * int(eu.numel()) + 8 * n
    return total


def read_traffic(expect_hash):
    """HBM bytes per k_isect launch from the committed counter summary, or
    None when it is missing or was taken on other kernel sources."""
    if not os.path.exists(TRAFFIC_SUMMARY):
        return None
    kv = {}
    with open(TRAFFIC_SUMMARY) as f:
        for line in f:
            m = re.match(r"^([a-z_0-9]+) = (\S+)\s*$", line)
            if m:
                kv[m.group(1)] = m.group(2)
    try:
        if kv["kernel_source_sha256"] != expect_hash:
            return None
        return float(kv["isect_hbm_bytes"])
    except (KeyError, ValueError):
        return None


def golden(name):
    """(n, m, T, T0, T1, |E0|) the oracle stored for a large graph, or None."""
    with open(GOLDEN) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                parts = line.split()
                if parts[0] == name:
                    return tuple(int(x) for x in parts[1:])
    return None


def copy_probe(torch):
    """A plain device pass of known size (read 1 GiB, write 1 GiB) for scaling
    the byte counters; its kernel (bitwise not over int32) runs nowhere else
    in this program, so a profile names it unambiguously.  Returns the best
    of the three passes in GB/s (bytes read + written over the HIP-event
    time): the bandwidth a streaming kernel reaches on this device."""
    a = torch.ones(COPY_PROBE_BYTES // 4, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    best = 0.0
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        torch.bitwise_not(a, out=b)
        e1.record()
        e1.synchronize()
        best = max(best, 2 * COPY_PROBE_BYTES / (e0.elapsed_time(e1) * 1e-3) / 1e9)
    print(f"# copy probe: 3 passes of {COPY_PROBE_BYTES} bytes read + written, best {best:.0f} GB/s",
          file=sys.stderr, flush=True)
    del a, b
    return best


def log(msg):
    print("# " + msg, file=sys.stderr, flush=True)


def make_graph(tc, torch, kind, size, seed):
    import graphgen
    if kind == "kronecker":
        n, s, d = graphgen.kronecker(size, 16, seed=seed)
    else:
        n, s, d = graphgen.chung_lu(1 << size, 2.1, 32.0, float(1 << 17), seed=seed)
    rp, col = tc.build_csr(n, torch.from_numpy(s).cuda(), torch.from_numpy(d).cuda())
    del s, d
    return n, rp, col


def timed_steps(counter, rp, col, steps, warmup, levels=None):
    """Mean wall time per step (seconds) and the per-step results."""
    import torch
    for _ in range(warmup):
        counter(rp, col, levels)
    torch.cuda.synchronize()
    results = []
    t0 = time.perf_counter()
    for _ in range(steps):
        results.append(counter(rp, col, levels))
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, results


def time_calls(fn, steps, warmup):
    """Mean wall time per call (seconds) of fn() and its last result."""
    import torch
    for _ in range(max(warmup, 1)):
        out = fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, out


def phase_means(results):
    return {k: float(np.mean([x.ms[k] for x in results])) for k in ("bfs", "partition", "bucket", "isect")}


def exact_vs_golden(name, n, m, r):
    g = golden(name)
    if g is None:
        return None
    return g == (n, m, r.T, r.T0, r.T1, r.e0)


def train_schedule(tc, torch, path, steps):
    """Measure the training graphs bucket by bucket, train the network, and
    store it with its training ranges and the measurements behind it."""
    from paper_2309_09064_amd import sched
    t0 = time.perf_counter()
    train = []
    for kind, size, seed in TRAIN_GRAPHS:
        _, rp, col = make_graph(tc, torch, kind, size, seed)
        lev, _ = tc.bfs_levels(rp, col)
        train.append((rp, col, lev))
    net, ms, losses, hull = sched.learn_marginal(train, steps=steps, log=log)
    changes = [{"graph": int(g), "kind": int(x[2]), "ob": int(x[0]), "pb": int(x[1]), "strategy": int(c),
                "delta_ms": round(float(d), 4), "spread_ms": round(float(sp), 4), "share": round(float(w), 4)}
               for g, x, c, d, sp, w in zip(ms.graph, ms.X, ms.c, ms.delta_ms, ms.spread_ms, ms.w) if d != 0.0]
    # the network's table (one table: it depends on the options only), then
    # each class of change it makes is kept only where the training graphs'
    # passes measure faster with it; the others are vetoed
    rp0, col0, _ = train[0]
    proposed = sched.learned_table(net, rp0.numel() - 1, col0.numel(), hull, SCHED_MARGIN)
    heur = tc.schedule_table(rp0.numel() - 1, col0.numel()).cpu().numpy()
    verified, vinfo = sched.verify_schedule(train, proposed)
    veto = sorted(set(sched.changed_classes(heur, proposed.cpu().numpy())) -
                  set(sched.changed_classes(heur, verified.cpu().numpy())))
    final = sched.learned_table(net, rp0.numel() - 1, col0.numel(), hull, SCHED_MARGIN, veto=veto)
    isect = {"heuristic": [sched.isect_ms([g], None) for g in train],
             "network": [sched.isect_ms([g], proposed.cpu().numpy()) for g in train],
             "learned": [sched.isect_ms([g], final.cpu().numpy()) for g in train]}
    meta = {"train_graphs": [f"{k} {'scale' if k == 'kronecker' else 'n = 2^'}{s}, seed {sd}"
                             for k, s, sd in TRAIN_GRAPHS],
            "target": "sign(t) log2(1 + |t|), t = pass-time change in ps per probe element",
            "rows": int(len(ms.c)), "steps": steps, "final_loss": float(losses[-1]),
            "train_heuristic_ms": ms.base_ms,
            "train_buckets_changed": {"network": int((proposed.cpu().numpy() != heur).sum()),
                                      "learned": int((final.cpu().numpy() != heur).sum())},
            "train_isect_ms": isect,
            "device": torch.cuda.get_device_name(0), "measured_changes": changes,
            "seconds": round(time.perf_counter() - t0, 1)}
    sched.save_net(path, net, hull, SCHED_MARGIN, meta, veto)
    log(f"schedule network written to {path}: {meta['rows']} rows, loss {meta['final_loss']:.3f}, "
        f"changed buckets on the training graphs {meta['train_buckets_changed']}")


def learned_leg(tc, torch, n, rp, col, T, steps, warmup):
    """Steps under the heuristic, the learned table (the stored network's
    choices minus the vetoed classes) and the network's own table,
    alternating; counts must equal T."""
    from paper_2309_09064_amd import sched
    if not os.path.exists(SCHED_NET):
        return {"error": f"{os.path.relpath(SCHED_NET, ROOT)} missing (bench.py --train-schedule writes it)"}
    net, hull, margin, doc = sched.load_net(SCHED_NET)
    nnz = col.numel()
    veto = [tuple(c) for c in doc.get("veto", [])]
    table = sched.learned_table(net, n, nnz, hull, margin, veto=veto)
    own = sched.learned_table(net, n, nnz, hull, margin)
    heur = tc.schedule_table(n, nnz)
    changed = int((table != heur).sum())
    out = {"network": os.path.relpath(SCHED_NET, ROOT), "train_graphs": doc["train_graphs"],
           "margin": margin, "vetoed_classes": [list(c) for c in veto], "buckets_changed": changed,
           "network_table_buckets_changed": int((own != heur).sum())}
    counters = {"heuristic": tc.Counter(n, nnz, tc.Options(timing=True))}
    if changed:
        counters["learned"] = tc.Counter(n, nnz, tc.Options(timing=True, sched_table=table))
    if out["network_table_buckets_changed"] and not torch.equal(own, table):
        counters["network_table"] = tc.Counter(n, nnz, tc.Options(timing=True, sched_table=own))
    if len(counters) > 1:
        for c in counters.values():
            for _ in range(warmup):
                c(rp, col)
        wall = {k: [] for k in counters}
        res = {k: [] for k in counters}
        for _ in range(steps):
            for k, c in counters.items():
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                r = c(rp, col)
                wall[k].append(time.perf_counter() - t0)
                res[k].append(r)
        for k in counters:
            assert all(x.T == T for x in res[k]), f"{k} schedule changed the count"
            out[k] = {"ms_per_step": 1e3 * float(np.mean(wall[k])), "phase_ms": phase_means(res[k])}
    h = out.get("heuristic", {}).get("ms_per_step")
    gain = h / out["learned"]["ms_per_step"] if "learned" in out else 1.0
    if "network_table" in out:
        out["network_table"]["speedup_vs_heuristic"] = h / out["network_table"]["ms_per_step"]
    out.update({"speedup_vs_heuristic": gain, "identical_to_heuristic": changed == 0,
                "target_met": gain > 1 + GAIN_NOISE})
    return out


def cpu_baseline(rp, col, seconds):
    """The oracle's edge iterator on a bounded sample of this graph's edges,
    on every host core it may use."""
    import oracle
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    g = oracle.as_csr(rp.numel() - 1, rp.cpu().numpy().astype(np.int64), col.cpu().numpy())
    nnz = g.nnz
    order = np.random.default_rng(0).permutation(CPU_SLICE)
    done, T_part, t_used = 0, 0, 0.0
    for off in order:
        es = np.arange(int(off), nnz, CPU_SLICE, dtype=np.int64)
        t0 = time.perf_counter()
        T_part += oracle.count_emd_entries(g, es, threads)
        t_used += time.perf_counter() - t0
        done += 1
        if t_used >= seconds:
            break
    frac = done / CPU_SLICE
    est = t_used / frac
    return {"value": g.m / est, "unit": "input edges/s", "cores": threads, "kind": "oracle",
            "sample": f"{done} interleaved slices of 1/{CPU_SLICE} of the CSR entries (every {CPU_SLICE}th "
                      f"entry from a random offset; {100 * frac:.2f} % of the edges) of the headline graph "
                      f"through the oracle's sorted-merge edge iterator (C, gcc -O2, OpenMP over entries, "
                      f"{threads} threads): {t_used:.1f} s, scaled by {1 / frac:.1f} to {est:.1f} s for the "
                      f"whole graph",
            "sample_T_estimate": int(round(T_part / frac))}


def cpu_alg4_context(n, rp, col):
    """Second stated CPU figure: the oracle's serial BFS levels + the counts of
    Algorithm 4 on one whole graph, one thread."""
    import oracle
    g = oracle.as_csr(n, rp.cpu().numpy().astype(np.int64), col.cpu().numpy())
    t0 = time.perf_counter()
    lev, _ = oracle.bfs_levels(g)
    r = oracle.alg4(g, lev)
    dt = time.perf_counter() - t0
    return {"value": g.m / dt, "unit": "input edges/s", "cores": 1, "seconds": dt, "T": r.T,
            "what": "oracle serial BFS levels + Algorithm 4's T0 and T1 (C, gcc -O2, one thread), whole graph"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--scale", type=int, default=24)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline legs")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-schedule legs")
    ap.add_argument("--no-secondary", action="store_true", help="skip the Chung-Lu, scale-20 and batch legs")
    ap.add_argument("--main-only", action="store_true",
                    help="time only the headline leg, so that a profile of the run holds its kernels alone")
    ap.add_argument("--batch-only", action="store_true",
                    help="time only the 4096-graph batch leg and print its record (for a profile of the batch)")
    ap.add_argument("--train-schedule", metavar="PATH",
                    help="measure the training graphs, train the schedule network, write it to PATH and exit")
    ap.add_argument("--train-steps", type=int, default=3000)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus above 1 is not supported "
                                   "(the multi-GPU sharding is described, not built)"}))
        sys.exit(2)
    if args.main_only:
        args.no_cpu = args.no_learned = args.no_secondary = True

    import torch
    import paper_2309_09064_amd as tc

    torch.cuda.set_device(0)
    # a streaming pass of known size: the bandwidth a plain kernel reaches
    # here, and the calibration of the byte counters in a profile of this run
    stream_gbs = copy_probe(torch)
    if args.train_schedule:
        train_schedule(tc, torch, args.train_schedule, args.train_steps)
        return
    if args.batch_only:
        print(json.dumps({"batch4096": batch_leg(tc, torch, args)}))
        return
    n, rp, col = make_graph(tc, torch, "kronecker", args.scale, args.seed)
    nnz = col.numel()
    m = nnz // 2
    log(f"graph: kronecker scale {args.scale} seed {args.seed}, n={n}, m={m}")

    # TC_TIMING makes the library record HIP events around each phase on the
    # stream it launches on; the cost is a few event records per step
    counter = tc.Counter(n, nnz, tc.Options(timing=True))
    step_s, results = timed_steps(counter, rp, col, args.steps, args.warmup)
    assert len({r.T for r in results}) == 1, "count changed between steps"
    r = results[-1]
    T = r.T
    ms = phase_means(results)
    log(f"timed: {args.steps} steps, {step_s * 1e3:.3f} ms/step, T={T}; phase ms {ms}")
    exact = exact_vs_golden(f"kronecker{args.scale}", n, m, r) if args.seed == 1 else None

    lev, _ = tc.bfs_levels(rp, col)
    balg = b_alg(rp, col, lev)
    # the library's own element count gives the same figure: 4 B per probe
    # element, the owner lists (every vertex's N1 and N0+ once), the records
    balg_lib = 4 * r.probes + 4 * (nnz - r.e0) + 8 * r.e0 + 8 * n
    assert balg == balg_lib, (balg, balg_lib)
    del lev
    torch.cuda.empty_cache()
    achieved = balg / (ms["isect"] * 1e-3) / 1e9
    default_workload = args.scale == 24 and args.seed == 1
    traffic = read_traffic(kernel_source_hash()) if default_workload else None
    log(f"k_isect: B_alg={balg / 1e9:.3f} GB in {ms['isect']:.3f} ms -> {achieved:.0f} GB/s; traffic {traffic}")

    learned = None
    secondary = {}
    if not args.no_learned:
        learned = learned_leg(tc, torch, n, rp, col, T, args.steps, args.warmup)
        log(f"learned: {json.dumps({k: v for k, v in learned.items() if k not in ('train_graphs',)})}")

    if not args.no_secondary:
        secondary = secondary_legs(tc, torch, args)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(rp, col, CPU_SECONDS)
        log(f"cpu baseline: {cpu['sample']}")
        if not args.no_secondary:
            n20, rp20, col20 = make_graph(tc, torch, "kronecker", 20, 1)
            cpu["alg4_serial_kronecker20"] = cpu_alg4_context(n20, rp20, col20)
            del rp20, col20

    out = {
        "metric": METRIC,
        "value": m / step_s,
        "unit": "input edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"kronecker scale {args.scale} edgefactor 16 (A,B,C,D=.57,.19,.19,.05), "
                               f"seed {args.seed}, int32 CSR, heuristic schedule",
                   "n": n, "m": m, "triangles": T, "T0": r.T0, "T1": r.T1, "e0": r.e0,
                   "k_percent": round(100.0 * r.e0 / m, 2), "levels": r.levels, "counts_bit_exact": exact,
                   "phase_ms": ms, "items": r.items, "strategy_items": r.strategy_items,
                   "learned_schedule": learned, "secondary": secondary},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": "k_isect",
                     "bytes_per_launch": balg, "ms_per_launch": ms["isect"],
                     "device_stream_gbs": stream_gbs},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


def secondary_legs(tc, torch, args):
    out = {}
    # Chung-Lu 2^22 (power law): heuristic, and the learned table
    n, rp, col = make_graph(tc, torch, "chunglu", 22, 1)
    m = col.numel() // 2
    c = tc.Counter(n, col.numel(), tc.Options(timing=True))
    st, res = timed_steps(c, rp, col, args.steps, args.warmup)
    r = res[-1]
    cl = {"workload": "chung-lu n=2^22, gamma 2.1, mean degree 32, max expected degree 2^17, seed 1",
          "value": m / st, "ms_per_step": st * 1e3, "phase_ms": phase_means(res), "m": m, "triangles": r.T,
          "counts_bit_exact": exact_vs_golden("chunglu22", n, m, r)}
    if not args.no_learned:
        cl["learned_schedule"] = learned_leg(tc, torch, n, rp, col, r.T, args.steps, args.warmup)
    out["chunglu22"] = cl
    log(f"chung-lu 2^22: {st * 1e3:.3f} ms/step")
    del rp, col
    torch.cuda.empty_cache()

    # Kronecker scale 20: the heuristic step and the paper's comparison legs
    n, rp, col = make_graph(tc, torch, "kronecker", 20, 1)
    m = col.numel() // 2
    c = tc.Counter(n, col.numel(), tc.Options(timing=True))
    st, res = timed_steps(c, rp, col, args.steps, args.warmup)
    r = res[-1]
    T = r.T
    k20 = {"workload": "kronecker scale 20 edgefactor 16, seed 1", "value": m / st, "ms_per_step": st * 1e3,
           "phase_ms": phase_means(res), "m": m, "triangles": T,
           "counts_bit_exact": exact_vs_golden("kronecker20", n, m, r)}
    # the same kernels with every edge horizontal (L = 0): plain forward-hashed
    # counting of the whole graph, no BFS (the paper's FH comparison)
    zero = torch.zeros(n, dtype=torch.int32, device="cuda")
    fs, fres = timed_steps(tc.Counter(n, col.numel(), tc.Options(timing=True)), rp, col, args.steps, args.warmup,
                           levels=zero)
    assert all(x.T == T for x in fres), "forward-hashed count differs"
    k20["forward_hashed_same_kernels"] = {"value": m / fs, "ms_per_step": fs * 1e3, "phase_ms": phase_means(fres)}
    # Algorithm 4 with the horizontal edges oriented by id (u < v as printed)
    # instead of by (degree, id) rank
    os_, ores = timed_steps(tc.Counter(n, col.numel(), tc.Options(timing=True, orientation=tc.TC_ORIENT_ID)), rp,
                            col, args.steps, args.warmup)
    assert all((x.T, x.T0, x.T1) == (T, r.T0, r.T1) for x in ores), "id-oriented count differs"
    k20["id_orientation"] = {"value": m / os_, "ms_per_step": os_ * 1e3, "phase_ms": phase_means(ores)}
    for name, fn in (("vertex_triangles", tc.vertex_triangles), ("edge_support", tc.edge_support)):
        x_s, (_, rx) = time_calls(lambda: fn(rp, col), args.steps, args.warmup)
        assert rx.T == T, f"{name} count differs"
        k20[name] = {"value": m / x_s, "ms_per_step": x_s * 1e3}
    ce_s, rce = time_calls(lambda: tc.count_cover_edge(rp, col), args.steps, args.warmup)
    rl_s, (rp2, col2, _) = time_calls(lambda: tc.relabel_by_degree(rp, col), args.steps, args.warmup)
    bd_s, rbd = time_calls(lambda: tc.count(rp2, col2), args.steps, args.warmup)
    ced_s, rced = time_calls(lambda: tc.count_cover_edge(rp2, col2), args.steps, args.warmup)
    assert rce.T == T and rbd.T == T and rced.T == T, "a variant's count differs"
    k20["paper_variants"] = {
        "cover_edge_alg3": {"ms_per_step": ce_s * 1e3, "value": m / ce_s},
        "degree_relabel_ms": rl_s * 1e3,
        "baderd": {"ms_per_step": (rl_s + bd_s) * 1e3, "value": m / (rl_s + bd_s), "count_ms": bd_s * 1e3,
                   "k_percent": round(100.0 * rbd.e0 / m, 2)},
        "ced": {"ms_per_step": (rl_s + ced_s) * 1e3, "value": m / (rl_s + ced_s), "count_ms": ced_s * 1e3}}
    out["kronecker20"] = k20
    log(f"kronecker 20: {st * 1e3:.3f} ms/step; id orientation {os_ * 1e3:.3f}; forward-hashed {fs * 1e3:.3f}; "
        f"cover edge {ce_s * 1e3:.3f}")
    del rp, col, rp2, col2, zero
    torch.cuda.empty_cache()
    out["batch4096"] = batch_leg(tc, torch, args)
    return out


def batch_golden():
    counts = []
    with open(BATCH_GOLDEN) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                counts.append(int(line.split()[4]))
    return np.array(counts, dtype=np.int64)


def batch_leg(tc, torch, args):
    """The 4096-graph batch (half Erdos-Renyi, half Kronecker scale 8-16):
    tiles tuned on the disjoint union, then the eager batched call and the
    captured plan's replays, every count checked against the oracle's."""
    import concurrent.futures as cf
    import graphgen
    from paper_2309_09064_amd import autotune
    t0 = time.perf_counter()
    rec = graphgen.batch_recipe(4096, seed=0)
    with cf.ThreadPoolExecutor(16) as ex:
        parts = list(ex.map(graphgen.batch_member_tuples, rec))
    voff = np.concatenate([[0], np.cumsum([p[0] for p in parts])]).astype(np.int64)
    src = torch.from_numpy(np.concatenate([p[1] + np.int32(voff[i]) for i, p in enumerate(parts)])).cuda()
    dst = torch.from_numpy(np.concatenate([p[2] + np.int32(voff[i]) for i, p in enumerate(parts)])).cuda()
    del parts
    rp, col = tc.build_csr(int(voff[-1]), src, dst)
    del src, dst
    batch = tc.Batch.from_union(rp, col, voff)
    m = col.numel() // 2
    t_ready = time.perf_counter() - t0
    opts, rep = autotune.tune(rp, col, space=BATCH_TUNE_SPACE, repeats=1)
    opts.timing = False
    del rp, col
    torch.cuda.empty_cache()
    want = batch_golden()
    ws = tc.workspace(tc.batch_workspace_bytes(batch, opts))
    e_s, (counts, res) = time_calls(lambda: tc.count_batched(batch, options=opts, ws=ws), args.steps, args.warmup)
    eager_exact = bool(np.array_equal(counts.cpu().numpy(), want))
    del ws
    torch.cuda.empty_cache()
    t1 = time.perf_counter()
    plan = tc.BatchPlan(batch, opts)
    capture_s = time.perf_counter() - t1
    for _ in range(max(args.warmup, 1)):
        plan.launch()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(args.steps):
        got = plan.launch()
    torch.cuda.synchronize()
    r_s = (time.perf_counter() - t2) / args.steps
    replay_exact = bool(np.array_equal(got.cpu().numpy(), want))
    plan.close()
    log(f"batch: {len(rec)} graphs, m={m}: eager {e_s * 1e3:.2f} ms, captured replay {r_s * 1e3:.2f} ms "
        f"(capture {capture_s:.3f} s); counts exact {eager_exact and replay_exact}")
    return {"workload": "4096 graphs: 2048 Erdos-Renyi G(n, p), n log-uniform in [64, 65536], mean degree "
                        "U[8, 64]; 2048 Kronecker, scale U{8..16}, edgefactor 16; member i seeded 1000 + i",
            "graphs": len(rec), "vertices": int(voff[-1]), "m": m, "triangles": int(want.sum()),
            "counts_bit_exact": eager_exact and replay_exact, "graphs_checked": int(len(want)),
            "tuned": {k: getattr(opts, k) for k in autotune.TUNED_FIELDS}, "tune_report": rep,
            "eager": {"value": m / e_s, "ms_per_step": e_s * 1e3},
            "captured_replay": {"value": m / r_s, "ms_per_step": r_s * 1e3, "capture_s": capture_s},
            "prepare_s": t_ready}


if __name__ == "__main__":
    main()
