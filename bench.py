#!/usr/bin/env python3
"""Benchmark: exact h-motif / 3h-motif counting (MoCHy-E) on one MI355X.

--workload medium-exact (default) is described below; --workload large-aplus
times MoCHy-A+ on the large hypergraph without a stored line graph, and
--workload batched-cp the batched significance/CP call against sequential
calls, --workload serving a Poisson stream of CP requests through the
continuous-batching server (see the functions of the same names).

Workload: the medium synthetic hypergraph (20,000 nodes, 100,000 drawn
hyperedges, sizes 2..25 with P(s) ~ s^-2.5, Zipf(1.0) node popularity,
seed 1, duplicates removed).  Its CSR is resident in HBM before timing.

One step = the whole exact path on the device: validation, transpose, line
graph (Algorithm 1), per-neighbour region records, MoCHy-E pair enumeration
with classification into 26 h-motifs and 431 3h-motifs (Algorithm 2), the
light-node correction, and the 457 counts back on the host.

Prints one JSON line.  value = connected triples classified per second
(sum of all h-motif counts / step time).  The roofline object is for the pair
kernel (integer-ALU bound: algorithmic operations per pair of neighbour
groups against the integer VALU rate measured in the same run), timed with
HIP events on the stream it runs on; correction_roofline is the light-pair
fix kernel's (bytes against HBM).  The same line carries the batched CP
comparison (base + 64 copies at --scale, one call against 65 sequential
calls, identical counts) and a serving stream (--requests at --rate through
the continuous-batching server, p50/p99 latency), and the CPU baseline: the
oracle (plain MoCHy-E) on a degree-stratified sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PAIR_KERNEL_SRC = os.path.join(ROOT, "paper_2310_15668_amd", "csrc", "exact.hip")
COUNTERS_SUMMARY = os.path.join(ROOT, "profiles", "k_exact_grouped_medium_counters.md")
FIX_KERNEL_SRC = os.path.join(ROOT, "paper_2310_15668_amd", "csrc", "correct.hip")
FIX_SUMMARY = os.path.join(ROOT, "profiles", "k_light_fix_medium_counters.md")
# the on-the-fly enumeration phase: k_enum (free.hip), k_memo and k_msample
# (memo.hip), their shared walk (walk.h)
ENUM_SRCS = [os.path.join(ROOT, "paper_2310_15668_amd", "csrc", f) for f in ("free.hip", "memo.hip", "walk.h")]
ENUM_SUMMARY = os.path.join(ROOT, "profiles", "enum_phase_large_aplus.md")
WORKLOAD = ("medium exact MoCHy-E: 20000 nodes, 100000 drawn hyperedges (duplicates removed), "
            "sizes 2..25 P(s)~s^-2.5, Zipf(1.0) node popularity, seed 1")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def source_digest(paths):
    """sha256 of a source file, or of several files' contents in order."""
    import hashlib
    d = hashlib.sha256()
    for path in ([paths] if isinstance(paths, str) else paths):
        with open(path, "rb") as f:
            d.update(f.read())
    return d.hexdigest()


def summary_values(summary, source):
    """'- key: value' lines of a committed rocprofv3 summary, or None if it is
    missing or the kernel source changed since its counters were taken."""
    if not os.path.exists(summary):
        return None
    vals = {}
    with open(summary) as f:
        for line in f:
            if ":" in line and line.strip().startswith("- "):
                k, v = line.strip()[2:].split(":", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel_source_sha256") != source_digest(source):
        return None
    return vals


# Integer vector-ALU ceiling from the chip's unit counts: 256 CUs, each with
# 4 SIMD units of 16 lanes (one wave64 instruction per CU per cycle), at the
# 2.4 GHz peak engine clock: 39.3e12 32-bit lane instructions per second.  A
# pure integer-VALU kernel of the pair kernel's instruction mix
# (mochy_calibrate_valu) sustains about that on the box, so the roofline
# takes the measured rate, from the same run, as its peak.
NUM_CUS, CLOCK_HZ, LANES = 256, 2.4e9, 64
VALU_PEAK_DERIVED = NUM_CUS * LANES * CLOCK_HZ

# Algorithmic integer vector instructions per unit of the exact pair kernel
# (Lemma 2's region sizes from the two neighbours' records; counted as
# instructions, as the calibrated ceiling is, so a packed instruction that
# does two 16-bit operations counts once; the class-table read and the
# histogram add are LDS operations and not counted):
#  * a pair of neighbour groups that both have a member above the centre
#    (its class is needed in full): the three mask intersections (centre
#    nodes, two words of heavy outside nodes), three population counts with
#    their offsets added in the same instruction (t + 2, and R5 + 2 in two),
#    a shift-or packing t + 2 and R5 + 2 into the halves of one word, a
#    compare of that word for the disjointness test (t = R5 = 0), a
#    shift-add for 2 (|e_i| - |e_i ∩ e_k| + t), the seven ternary digits
#    max(2 - R, 0) as one saturating subtract and three packed ones (two
#    digits each), the base-3 code doubled into the table's byte offset as
#    three two-term dot products, the weight N_j N_k or A_j A_k as a select
#    of the lane's (0, N_k) or (A_k, 0) and a two-term dot product with j's
#    counts packed as 16-bit halves, and one add for the histogram address:
#    19 (21 where a row reaches 2^16 neighbours, the counts no longer fit 16
#    bits and the weight takes two selects and two multiplies for 48 bits);
#  * any other pair of groups (counted only when open): the centre-node
#    intersection, two AND-ORs for the heavy words, max(1 - x, 0) and a
#    multiply-add into the run's sum over disjoint groups: 5.
OPS_FULL_PAIR, OPS_OPEN_PAIR = 19, 5
WIDE_ROW = 1 << 16  # line-graph degree from which a pair weight takes 48 bits
# Algorithmic bytes of the light-pair fix kernel: the partner row's entry
# (4-byte hyperedge id) for every scanned entry, and for every centre it finds
# the partner row's 4-byte record mask and owner row's 2-byte size word.
FIX_BYTES_SCANNED, FIX_BYTES_CENTRE = 4, 6


def valu_issue(kernel_ms, ceiling):
    """The pair kernel's VALU wave-instructions per launch (SQ_INSTS_VALU from
    the committed counter summary) over this run's kernel time, per CU per
    cycle, beside the calibrated ceiling in the same unit; None if the
    counters are stale."""
    vals = summary_values(COUNTERS_SUMMARY, PAIR_KERNEL_SRC)
    if vals is None or "SQ_INSTS_VALU" not in vals:
        return None
    n = float(vals["SQ_INSTS_VALU"])
    rate = n / (NUM_CUS * CLOCK_HZ * kernel_ms * 1e-3)
    peak = ceiling / (LANES * NUM_CUS * CLOCK_HZ)
    return {"valu_wave_instructions_per_launch": n, "per_cu_per_cycle": rate,
            "calibrated_per_cu_per_cycle": peak, "frac": rate / peak,
            "source": "profiles/k_exact_grouped_medium_counters.md"}


def valu_calibration(M, ctx, iters=1 << 16, runs=3):
    """Best integer-VALU rate (lane instructions/s) of mochy_calibrate_valu."""
    best = 0.0
    for _ in range(runs):
        ms, ops = M.mochy_calibrate_valu(ctx, iters)
        best = max(best, ops / (ms * 1e-3))
    return best


def measured_traffic(summary=None, source=None):
    """HBM bytes per launch of a kernel from a committed rocprofv3 counter
    summary (default: the exact pair kernel's), or None if there is none or
    the kernel source changed since the counters were taken."""
    vals = summary_values(summary or COUNTERS_SUMMARY, source or PAIR_KERNEL_SRC)
    try:
        return float(vals["traffic_bytes_per_launch"]) if vals else None
    except (KeyError, ValueError):
        return None


def copy_calibration():
    """A plain device-to-device copy of 1 GiB, for scaling the byte counters."""
    import torch
    n = 1 << 30
    src = torch.empty(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty(n, dtype=torch.uint8, device="cuda")
    src.fill_(1)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n, "copies": 3}), flush=True)


def valu_calibration_runs():
    """mochy_calibrate_valu at 2^12, 2^14 and 2^16 rounds, one JSON line each
    (the integer VALU ceiling, for counter runs under rocprofv3)."""
    import paper_2310_15668_amd as M
    ctx = M.Context(0)
    try:
        for it in (1 << 12, 1 << 14, 1 << 16):
            ms, ops = M.mochy_calibrate_valu(ctx, it)
            rate = ops / (ms * 1e-3)
            print(json.dumps({"iters": it, "ms": ms, "lane_ops": ops, "lane_ops_per_s": rate,
                              "wave_instr_per_cu_per_cycle": rate / LANES / (NUM_CUS * CLOCK_HZ)}), flush=True)
    finally:
        ctx.close()


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(h, seconds):
    """The oracle (plain MoCHy-E, OpenMP over centres) timed on this host.

    Threads: every core this process may run on, within the host's share for
    one GPU (OMP_NUM_THREADS when set).  Medium sample: centres stratified by
    line-graph degree octave, each octave contributing candidates in
    proportion to its share of the whole workload's (hubs included, up to
    centres one core finishes within the time budget), largest first.  Also
    the whole tiny workload on one thread (the paper's default setting)."""
    import numpy as np
    from oracle import native
    from workloads import make_config
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    share = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    cores = max(1, min(avail, share) if share > 0 else avail)

    tiny = make_config("tiny")
    t0 = time.perf_counter()
    t26, _, _ = native.mochy_e(tiny, nthreads=1)
    t_tiny = time.perf_counter() - t0

    deg, _ = native.line_graph_degrees(h, cores)
    cand = deg * (deg - 1) // 2
    total = int(cand.sum())
    # per-core rate from a calibration run of mid-degree centres
    mid = np.nonzero((deg >= 1000) & (deg < 2000))[0]
    calib = mid[:: max(1, mid.size // (2 * cores))][: 2 * cores].astype(np.int64)
    t0 = time.perf_counter()
    native.mochy_e_centers(h, calib, nthreads=cores)
    rate_core = max(float(cand[calib].sum()) / ((time.perf_counter() - t0) * cores), 1e5)
    budget = rate_core * cores * seconds        # candidates the sample may hold
    cap = rate_core * seconds * 0.9             # one centre within the budget on one core
    octs = np.floor(np.log2(np.maximum(deg, 1))).astype(np.int64)
    chosen, rows = [], []
    for k in range(1, int(octs.max()) + 1):
        in_oct = np.nonzero((octs == k) & (cand > 0))[0]
        if in_oct.size == 0:
            continue
        want = budget * float(cand[in_oct].sum()) / total
        ok = in_oct[cand[in_oct] <= cap]
        if ok.size == 0:
            rows.append({"degrees": [int(2 ** k), int(2 ** (k + 1) - 1)],
                         "workload_share": float(cand[in_oct].sum()) / total, "centres": 0,
                         "sampled_candidates": 0})
            continue
        n = int(min(ok.size, max(1, round(want / float(cand[ok].mean())))))
        pick = ok[np.linspace(0, ok.size - 1, n).round().astype(np.int64)]
        pick = np.unique(pick)
        chosen.append(pick)
        rows.append({"degrees": [int(2 ** k), int(2 ** (k + 1) - 1)],
                     "workload_share": float(cand[in_oct].sum()) / total, "centres": int(pick.size),
                     "sampled_candidates": int(cand[pick].sum())})
    centres = np.concatenate(chosen)
    centres = centres[np.argsort(-cand[centres], kind="stable")]  # largest start first
    t0 = time.perf_counter()
    c26, _, _ = native.mochy_e_centers(h, centres, nthreads=cores)
    dt = time.perf_counter() - t0
    tri, nc = int(c26.sum()), int(cand[centres].sum())
    sampled_share = sum(r["workload_share"] for r in rows if r["centres"])
    return {
        "value": tri / dt, "unit": "triples/s", "cores": cores, "kind": "oracle",
        "sample": f"{centres.size} medium centres stratified by line-graph degree octave (each octave's "
                  f"candidates in proportion to its share of the workload; octaves holding "
                  f"{100 * sampled_share:.1f} % of the candidates represented, hubs up to degree "
                  f"{int(deg[centres].max())}): {nc} MoCHy-E candidates ({100.0 * nc / total:.3f} % of "
                  f"the workload), {tri} connected triples attributed to them, {dt:.1f} s wall",
        "candidates_per_s": nc / dt,
        "extrapolated_medium_s": total / (nc / dt),
        "nproc": os.cpu_count(), "affinity_cores": avail, "cpu_model": cpu_model(),
        "octaves": rows,
        "tiny_one_thread": {"value": int(t26.sum()) / t_tiny, "unit": "triples/s", "seconds": t_tiny,
                            "connected_triples": int(t26.sum()), "threads": 1},
    }


def device_csr(h):
    import torch
    return (torch.from_numpy(h.edge_ptr).cuda(), torch.from_numpy(h.edge_nodes).cuda(), h.num_nodes)


def large_aplus(args):
    """MoCHy-A+ on the large hypergraph without a stored line graph: one step =
    projection (validation, transpose, per-slot node lists, degrees, hyperwedge
    order) + r samples (draw, group by row, pick e_j; group by key hyperedge,
    memoize the keys' neighbourhood counts, enumerate each sample's other side)."""
    import numpy as np
    import torch
    import paper_2310_15668_amd as M
    from paper_2310_15668_amd import _lib
    from workloads import make_config

    h = make_config("large")
    log(f"workload |E|={h.num_edges} |V|={h.num_nodes} nnz={h.nnz}")
    dp, dn, V = device_csr(h)
    torch.cuda.synchronize()
    ctx = M.Context(0, torch.cuda.current_stream().cuda_stream)
    g = M.mochy_project(ctx, dp, dn, V)
    W = g.num_hyperwedges
    st = M.mochy_graph_stats(ctx, g)
    g.close()
    r = args.samples if args.samples else W * 5 // 100
    log(f"|wedges|={W} r={r} ({100.0 * r / W:.3g}% of the hyperwedges)")
    for w in range(args.warmup):
        log(f"warmup {w + 1}/{args.warmup}")
        g = M.mochy_project(ctx, dp, dn, V)
        M.mochy_count_sampled(ctx, g, min(r, 1 << 22), args.seed)
        g.close()
    phase_sum = {k: 0.0 for k in _lib.PHASES}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        log(f"step {s + 1}/{args.steps}")
        g = M.mochy_project(ctx, dp, dn, V)
        for k, v in M.mochy_phase_ms(ctx).items():
            phase_sum[k] += v
        # samples [0, r) in calls of at most 2^28 (consecutive Philox counters,
        # so the hits add up to one call's); est = hits * |wedges| / (w * r)
        raw26 = np.zeros(26, dtype=np.int64)
        est26 = np.zeros(26)
        memo = {"samples": 0, "memo_samples": 0, "memo_keys": 0, "memo_walk": 0}
        for n0 in range(0, r, 1 << 28):
            rr = min(1 << 28, r - n0)
            c26, e26, _, _ = M.mochy_count_sampled(ctx, g, rr, args.seed, n0)
            raw26 += c26
            est26 += e26 * (rr / r)
            for k, v in M.mochy_phase_ms(ctx).items():
                phase_sum[k] += v
            for k, v in M.mochy_memo_stats(ctx).items():
                if k in memo:
                    memo[k] += v
            log(f"  samples {n0 + rr}/{r}")
        g.close()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.close()
    K = max(args.steps, 1)
    pairs = int(raw26.sum())
    enum_ms = phase_sum["sample_enum"] / K
    model = 24  # bytes per (sample, e_k) pair: 16 + 4 * min size, sizes >= 2
    # the key memos stand for most pairs through (size, overlap) counts, so
    # the per-pair model overstates the bytes moved; the roofline takes the
    # measured HBM-side bytes of a 2^27-sample chunk (committed counters),
    # scaled to this run's samples, or none if the kernels changed since
    chunk_bytes = measured_traffic(ENUM_SUMMARY, ENUM_SRCS)
    moved = chunk_bytes * (r / float(1 << 27)) if chunk_bytes else None
    achieved = moved / (enum_ms * 1e-3) / 1e9 if moved else None
    out = {
        "metric": "(sample, e_k) pairs classified/s (MoCHy-A+)",
        "value": pairs / (dt / K), "unit": "pairs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3 / K,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": "large sampled MoCHy-A+: 1,000,000 nodes, 2,000,000 drawn hyperedges "
                               "(duplicates removed), sizes 2..25 P(s)~s^-2.8, Zipf(0.9), seed 2; "
                               "no stored line graph",
                   "hyperedges": st["num_edges"], "hyperwedges": W, "samples": r,
                   "sample_fraction": r / W, "seed": args.seed, "max_line_degree": st["max_line_degree"],
                   "samples_per_s": r / (dt / K), "estimated_connected_triples": float(est26.sum()),
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm",
                     "kernel": "enumeration phase: k_memo + k_msample, k_enum for keys left without a memo",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS if achieved else None,
                     "traffic": chunk_bytes,
                     "traffic_launch": "one chunk of 2^27 samples",
                     "achieved_from": "measured FETCH_SIZE + WRITE_SIZE per chunk (profiles/enum_phase_large_aplus.md) "
                                      "x samples / 2^27, over the phase time",
                     "model": "16 + 4*min(|e_i|,|e_j|,|e_k|) >= 24 bytes per (sample, e_k) pair "
                              "(model_bytes_per_s; memoized pairs are never read one by one)",
                     "model_bytes_per_s": model * pairs / (enum_ms * 1e-3),
                     "kernel_ms": enum_ms, "pairs_per_s": pairs / (enum_ms * 1e-3)},
        "phases_ms": {k: v / K for k, v in phase_sum.items() if v},
        "key_memos": {"memo_sample_share": memo["memo_samples"] / max(memo["samples"], 1),
                      "keys_memoized": memo["memo_keys"], "memo_walk_entries": memo["memo_walk"]},
    }
    print(json.dumps(out), flush=True)


def run_batched(scale, steps=1, warmup=1, tune=False):
    """One mochy_profile call over the batched base hypergraph and its 64
    stub-matched copies, against 65 sequential project + count calls on the
    same context (identical counts required); best of `steps` each."""
    import numpy as np
    import torch
    import paper_2310_15668_amd as M
    from workloads import make_config, stub_matching_copy
    from workloads.generators import BATCHED_COPY_SEEDS

    base = make_config("batched_base", scale=scale)
    graphs = [base] + [stub_matching_copy(base, s) for s in BATCHED_COPY_SEEDS]
    log(f"batched CP at scale {scale}: base |E|={base.num_edges}, {len(graphs)} graphs, "
        f"{sum(g.num_edges for g in graphs)} hyperedges in all")
    dev = [device_csr(g) for g in graphs]
    torch.cuda.synchronize()
    ctx = M.Context(0, torch.cuda.current_stream().cuda_stream)
    big = scale >= 0.5  # calls of minutes: progress lines (the library's per sub-batch lines too)
    if big:
        os.environ["MOCHY_LOG_BATCHES"] = "1"

    def sequential():
        rows = []
        for x, (p, n, V) in enumerate(dev):
            g = M.mochy_project(ctx, p, n, V)
            c26, c431 = M.mochy_count_exact(ctx, g)
            g.close()
            rows.append(np.concatenate([c26, c431]))
            if big and (x + 1) % 8 == 0:
                log(f"  sequential: {x + 1}/{len(dev)} graphs counted")
        return np.array(rows)

    for w in range(warmup):
        log(f"batched warmup {w + 1}/{warmup}")
        M.mochy_profile(ctx, dev[:3])
    tuned = None
    if tune:  # the pair kernel's launch shape, timed on this batch (untimed here)
        from paper_2310_15668_amd.tune import tune_batch
        log("tuning the pair kernel's launch shape on the batch")
        res = tune_batch(ctx, dev)
        tuned = {"batch_launch": res["launch"], "pair_blocks_per_cu": res["blocks"],
                 "pair_ms": {f"launch={a},blocks={b}": t for (a, b), t in res["times"].items()}}
        log(f"tuned: {tuned}")
    times_b, times_s = [], []
    for s in range(steps):
        log(f"batched step {s + 1}/{steps}: one call")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        counts, sig26, cp26, sig431, cp431 = M.mochy_profile(ctx, dev)
        torch.cuda.synchronize()
        times_b.append(time.perf_counter() - t0)
        batches = M.mochy_exact_stats(ctx)["profile_batches"]
        log(f"batched step {s + 1}/{steps}: 65 sequential calls")
        t0 = time.perf_counter()
        seq = sequential()
        torch.cuda.synchronize()
        times_s.append(time.perf_counter() - t0)
        if not (seq == counts).all():
            raise SystemExit("batched and sequential counts differ")
    ctx.close()
    tb, ts = min(times_b), min(times_s)
    triples = int(counts[:, :26].sum())
    out = {"speedup": ts / tb, "batched_s": tb, "sequential_s": ts, "graphs": len(graphs),
           "sub_batches": batches,
           "scale": scale, "base_hyperedges": base.num_edges,
           "hyperedges_all_graphs": int(sum(g.num_edges for g in graphs)),
           "connected_triples_all_graphs": triples, "batched_triples_per_s": triples / tb,
           "sequential_triples_per_s": triples / ts, "identical_counts": True, "steps": steps,
           "workload": f"batched CP: base hypergraph (50,000 nodes, 150,000 drawn hyperedges, sizes 2..20 "
                       f"P(s)~s^-2.5, Zipf(1.1), seed 3) and 64 stub-matched copies (seeds 100..163), "
                       f"nodes and hyperedges scaled by {scale}; one mochy_profile call against 65 "
                       f"sequential project + count calls on one context"}
    if tuned is not None:
        out["tuned"] = tuned
    return out


def batched_cp(args):
    """Significance and CP of the batched base hypergraph against 64
    stub-matched copies: one mochy_profile call (all 65 graphs projected and
    counted together) versus 65 sequential project + count calls."""
    res = run_batched(args.scale, args.steps, args.warmup, args.tune)
    out = {
        "metric": "batched CP speedup over 65 sequential project+count calls",
        "value": res["speedup"], "unit": "x", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": res["batched_s"] * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": res["workload"], "scale": args.scale, "graphs": res["graphs"],
                   "parallelism": "single GPU"},
        "batched": res,
    }
    print(json.dumps(out), flush=True)


def run_serving(requests, rate, max_edges, slots_list, log_every=None):
    """A Poisson stream of CP requests (a hypergraph + 8 stub-matched copies
    each) through the continuous-batching server, once per slot count;
    answers must not depend on the slot count."""
    import numpy as np
    import torch
    from paper_2310_15668_amd.serving import CPServer
    from workloads import poisson_arrivals, serving_copies, serving_request

    log_every = log_every or max(1, min(50, requests // 10))
    log(f"generating {requests} requests (|E| log-uniform in [1000, {max_edges}], 8 copies each)")
    reqs, sizes = [], []
    for n in range(requests):
        h = serving_request(n, 1000, max_edges)
        sizes.append(h.num_edges)
        reqs.append([(g.edge_ptr, g.edge_nodes, g.num_nodes) for g in [h] + serving_copies(n, h, 8)])
    arrivals = poisson_arrivals(requests, rate)
    torch.cuda.init()
    runs, answers = {}, {}
    for slots in slots_list:
        with CPServer(0, slots=slots) as srv:
            for t in [srv.submit(r) for r in reqs[:2]]:  # warm-up
                t.wait()
            t0 = time.perf_counter()
            tickets = []
            for n, r in enumerate(reqs):
                delay = t0 + arrivals[n] - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
                tickets.append(srv.submit(r, arrival=t0 + arrivals[n]))
            for k, t in enumerate(tickets):
                t.wait()
                if (k + 1) % log_every == 0:
                    log(f"  slots={slots}: {k + 1}/{len(tickets)} answered")
            end = max(t.done for t in tickets)
        lat = np.array([t.latency for t in tickets])
        answers[slots] = [t.result["counts"] for t in tickets]
        triples = int(sum(a[:, :26].sum() for a in answers[slots]))
        runs[slots] = {"requests_per_s": len(tickets) / (end - t0), "p50_s": float(np.percentile(lat, 50)),
                       "p99_s": float(np.percentile(lat, 99)), "mean_s": float(lat.mean()),
                       "makespan_s": end - t0, "triples_per_s": triples / (end - t0)}
        log(f"slots={slots}: {runs[slots]}")
    first = answers[slots_list[0]]
    for slots in slots_list[1:]:
        if not all((a == b).all() for a, b in zip(first, answers[slots])):
            raise SystemExit("answers differ between the server configurations")
    return {"runs": runs, "median_edges": int(np.median(sizes)), "max_edges_drawn": int(max(sizes)),
            "workload": f"serving CP requests: {requests} hypergraphs, |E| log-uniform in [1000, {max_edges}], "
                        f"nodes 0.4|E|, sizes 2..25 P(s)~s^-2.5, Zipf(1.0), Poisson arrivals at {rate} req/s, "
                        f"each request = exact counts of the hypergraph and 8 stub-matched copies -> "
                        f"significance and CP"}


def serving(args):
    """CP requests arriving as a Poisson stream, served by the
    continuous-batching server with `slots` concurrent streams, and the same
    stream with one slot for comparison."""
    res = run_serving(args.requests, args.rate, args.max_edges, [args.slots, 1])
    best = res["runs"][args.slots]
    out = {
        "metric": "CP requests served/s (p50/p99 latency beside)",
        "value": best["requests_per_s"], "unit": "requests/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": best["makespan_s"] * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": res["workload"], "slots": args.slots, "median_edges": res["median_edges"],
                   "parallelism": "single GPU"},
        "p50_s": best["p50_s"], "p99_s": best["p99_s"],
        "continuous_batching": best, "one_slot": res["runs"][1],
        "answers_identical_across_configurations": True,
    }
    print(json.dumps(out), flush=True)


def tradeoff(args):
    """MoCHy-A (hyperedge samples) against MoCHy-A+ (hyperwedge samples) on
    the medium hypergraph: relative error of the estimates against the exact
    counts, and time, over a range of sample counts."""
    import numpy as np
    import torch
    import paper_2310_15668_amd as M
    from workloads import make_config

    h = make_config("medium")
    dp, dn, V = device_csr(h)
    torch.cuda.synchronize()
    ctx = M.Context(0, torch.cuda.current_stream().cuda_stream)
    g = M.mochy_project(ctx, dp, dn, V)
    exact, _ = M.mochy_count_exact(ctx, g)
    big = exact > 1e-3 * exact.sum()
    rows = []
    for name, fn, counts in (("A+", M.mochy_count_sampled, (10 ** 5, 10 ** 6, 10 ** 7, 10 ** 8)),
                             ("A", M.mochy_count_sampled_edges, (10, 100, 1000))):
        for n in counts:
            fn(ctx, g, min(n, 1000), 99)  # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, est26, _, _ = fn(ctx, g, n, args.seed)
            dt = time.perf_counter() - t0
            rel = np.abs(est26[big] - exact[big]) / exact[big]
            rows.append({"method": name, "samples": n, "seconds": dt, "max_rel_error": float(rel.max()),
                         "mean_rel_error": float(rel.mean())})
            log(rows[-1])
    g.close()
    ctx.close()
    out = {"metric": "relative error of motif-count estimates vs time (MoCHy-A and MoCHy-A+)",
           "value": None, "unit": "", "n_gpus": 1, "data": "synthetic", "dtype": "u32",
           "config": {"workload": "medium hypergraph (see medium-exact); h-motifs with at least 0.1 % "
                                  "of the connected triples", "seed": args.seed},
           "points": rows}
    print(json.dumps(out), flush=True)


def budget_sweep(args):
    """On-the-fly MoCHy-A+ with key memos (Algorithm 9) under memo budgets
    given as fractions of a stored line graph ((e_k, omega) entries of 8 bytes
    over both rows of every hyperwedge), the large hypergraph without a stored
    line graph: time per sample, the share of samples counted through a memo,
    and the same hits at every budget."""
    import numpy as np
    import torch
    import paper_2310_15668_amd as M
    from workloads import make_config

    name = args.sweep_graph
    h = make_config(name)
    dp, dn, V = device_csr(h)
    torch.cuda.synchronize()
    ctx = M.Context(0, torch.cuda.current_stream().cuda_stream)
    g = M.mochy_project(ctx, dp, dn, V, M.MOCHY_LG_FREE)
    W = g.num_hyperwedges
    lg_bytes = 2 * W * 8
    r = args.samples if args.samples else 1 << 25
    log(f"{name}: |E|={h.num_edges} |wedges|={W} r={r}; line graph as (e_k, omega) lists: {lg_bytes / 2**30:.1f} GiB")
    M.mochy_count_sampled(ctx, g, min(r, 1 << 20), 99)  # warm-up
    rows, ref = [], None
    for frac in (0.0, 1e-5, 1e-4, 1e-3, 1e-2):
        budget = min(int(frac * lg_bytes), 16 << 30)
        ctx.set_option(M.MOCHY_OPT_MEMO_BUDGET, budget)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        raw26, _, raw431, _ = M.mochy_count_sampled(ctx, g, r, args.seed)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ph = M.mochy_phase_ms(ctx)
        ms = M.mochy_memo_stats(ctx)
        if ref is None:
            ref = raw431
        rows.append({"budget_fraction_of_line_graph": frac, "budget_bytes": budget, "seconds": dt,
                     "samples_per_s": r / dt, "enum_ms": ph["sample_enum"], "draw_ms": ph["sample_draw"],
                     "memo_sample_share": ms["memo_samples"] / max(ms["samples"], 1),
                     "memo_keys": ms["memo_keys"], "arena_bytes_used": ms["arena_bytes"],
                     "same_hits": bool((raw431 == ref).all())})
        log(rows[-1])
    g.close()
    ctx.close()
    out = {"metric": "MoCHy-A+ samples/s vs key-memo budget (on-the-fly, Algorithm 9)",
           "value": None, "unit": "samples/s", "n_gpus": 1, "data": "synthetic", "dtype": "u32",
           "config": {"workload": f"{name} hypergraph, no stored line graph; one call of {r} samples",
                      "hyperwedges": W, "line_graph_list_bytes": lg_bytes, "seed": args.seed},
           "points": rows}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default 3; 1 for large-aplus)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="medium-exact",
                    choices=["medium-exact", "large-aplus", "batched-cp", "serving", "tradeoff", "budget"])
    ap.add_argument("--sweep-graph", default="large", choices=["medium", "large"],
                    help="budget: hypergraph of the memo-budget sweep")
    ap.add_argument("--samples", type=int, default=0,
                    help="large-aplus: samples per step (default 5%% of the hyperwedges)")
    ap.add_argument("--seed", type=int, default=2, help="large-aplus: Philox key")
    ap.add_argument("--scale", type=float, default=0.2,
                    help="batched-cp (and the batched part of medium-exact): scale of the base "
                         "hypergraph and its copies")
    ap.add_argument("--tune", action="store_true",
                    help="batched-cp: pick the pair kernel's launch shape by timing before the steps")
    ap.add_argument("--requests", type=int, default=200, help="serving: requests in the stream")
    ap.add_argument("--rate", type=float, default=50.0, help="serving: Poisson arrival rate (req/s)")
    ap.add_argument("--max-edges", type=int, default=20000,
                    help="serving: largest request (hyperedges; the stream's range is [1000, max])")
    ap.add_argument("--slots", type=int, default=4, help="serving: concurrent streams of the server")
    ap.add_argument("--cpu-seconds", type=float, default=30.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true",
                    help="medium-exact: leave out the batched CP comparison")
    ap.add_argument("--no-serving", action="store_true",
                    help="medium-exact: leave out the serving stream")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (counter calibration under rocprofv3)")
    ap.add_argument("--valu-calibration", action="store_true",
                    help="only run the integer VALU calibration kernel (its counters under rocprofv3)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: motifs are counted on one device "
              "(multi-GPU sharding is a design note only); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.steps is None:
        args.steps = 1 if args.workload == "large-aplus" else 3

    if args.copy_calibration:
        copy_calibration()
        return
    if args.valu_calibration:
        valu_calibration_runs()
        return
    if args.workload == "large-aplus":
        large_aplus(args)
        return
    if args.workload == "batched-cp":
        batched_cp(args)
        return
    if args.workload == "serving":
        serving(args)
        return
    if args.workload == "budget":
        return budget_sweep(args)
    if args.workload == "tradeoff":
        tradeoff(args)
        return
    medium_exact(args)


def medium_exact(args):
    """The default line: exact counts of the medium workload (value), the pair
    kernel's ALU roofline, the correction kernel's byte roofline, the oracle's
    CPU baseline, and the batched CP and serving measurements beside."""
    import numpy as np
    import torch
    import paper_2310_15668_amd as M
    from paper_2310_15668_amd import _lib
    from workloads import make_config

    h = make_config("medium")
    log(f"workload |E|={h.num_edges} |V|={h.num_nodes} nnz={h.nnz}")
    dev_ptr = torch.from_numpy(h.edge_ptr).cuda()
    dev_nodes = torch.from_numpy(h.edge_nodes).cuda()
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    ctx = M.Context(0, stream.cuda_stream)

    phase_sum = {k: 0.0 for k in _lib.PHASES}
    result = {}

    def step(record):
        g = M.mochy_project(ctx, dev_ptr, dev_nodes, h.num_nodes)
        ph = M.mochy_phase_ms(ctx)
        c26, c431 = M.mochy_count_exact(ctx, g)
        ph2 = M.mochy_phase_ms(ctx)
        if record:
            for k in phase_sum:
                phase_sum[k] += ph[k] + ph2[k]
        result["c26"], result["c431"] = c26, c431
        result["exact_stats"] = M.mochy_exact_stats(ctx)
        if "stats" not in result:
            result["stats"] = M.mochy_graph_stats(ctx, g)
        g.close()

    for w in range(args.warmup):
        log(f"warmup {w + 1}/{args.warmup}")
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        log(f"step {s + 1}/{args.steps}")
        step(True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    K = max(args.steps, 1)
    ms_step = dt * 1e3 / K
    log("integer VALU calibration")
    valu_peak = valu_calibration(M, ctx)
    ctx.close()

    c26 = result["c26"]
    st = result["stats"]
    xs = result["exact_stats"]
    triples = int(c26.sum())
    s_open = int(sum(c26[t - 1] for t in range(17, 23)))
    s_closed = triples - s_open
    identity_ok = (s_open + 3 * s_closed) == st["candidates"]

    pair_ms = phase_sum["exact_pairs"] / K
    ops_full = OPS_FULL_PAIR + (2 if st["max_line_degree"] >= WIDE_ROW else 0)
    ops = ops_full * xs["group_pairs_full"] + OPS_OPEN_PAIR * xs["group_pairs_open"]
    achieved = ops / (pair_ms * 1e-3)
    fix_ms = phase_sum["exact_fix_kernel"] / K
    fix_bytes = FIX_BYTES_SCANNED * xs["fix_scanned"] + FIX_BYTES_CENTRE * xs["fix_centres"]
    out = {
        "metric": "connected triples classified/s",
        "value": triples / (dt / K),
        "unit": "triples/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": WORKLOAD, "hyperedges": st["num_edges"], "nodes": st["num_nodes"],
                   "incidences": st["nnz"], "hyperwedges": st["hyperwedges"],
                   "max_line_degree": st["max_line_degree"], "candidates": st["candidates"],
                   "connected_triples": triples, "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "kernel": "k_exact_grouped (MoCHy-E pairs of neighbour groups)",
                     "achieved": achieved / 1e12, "peak": valu_peak / 1e12, "unit": "TOP/s",
                     "frac": achieved / valu_peak, "traffic": measured_traffic(),
                     "model": f"{ops_full} integer vector lane instructions per pair of neighbour groups "
                              f"classified in full, {OPS_OPEN_PAIR} per other pair (counted only when open)",
                     "peak_source": "integer VALU rate of mochy_calibrate_valu measured in this run "
                                    f"(chip-derived: 256 CUs x 64 lanes x 2.4 GHz = "
                                    f"{VALU_PEAK_DERIVED / 1e12:.1f} TOP/s)",
                     "peak_derived": VALU_PEAK_DERIVED / 1e12,
                     "kernel_ms": pair_ms, "group_pairs_full": xs["group_pairs_full"],
                     "group_pairs_open": xs["group_pairs_open"],
                     "candidates_per_s": st["candidates"] / (pair_ms * 1e-3),
                     "valu_issue": valu_issue(pair_ms, valu_peak)},
        "correction_roofline": {"bound": "hbm", "kernel": "k_light_fix (light-pair correction)",
                                "achieved": fix_bytes / (fix_ms * 1e-3) / 1e9 if fix_ms else None,
                                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                "frac": fix_bytes / (fix_ms * 1e-3) / 1e9 / HBM_PEAK_GBS if fix_ms else None,
                                "traffic": measured_traffic(FIX_SUMMARY, FIX_KERNEL_SRC),
                                "model": f"{FIX_BYTES_SCANNED} B per scanned row entry + {FIX_BYTES_CENTRE} B "
                                         "per centre examined",
                                "kernel_ms": fix_ms, "scanned_entries": xs["fix_scanned"],
                                "centres": xs["fix_centres"], "light_pairs": xs["light_pairs"]},
        "exact_stats": xs,
        "phases_ms": {k: v / K for k, v in phase_sum.items() if v},
        "identity_open_plus_3closed_eq_candidates": bool(identity_ok),
    }
    if not args.no_batched:
        log("batched CP comparison")
        out["batched_cp"] = run_batched(args.scale, steps=1, warmup=1)
    if not args.no_serving:
        log("serving stream")
        res = run_serving(args.requests, args.rate, args.max_edges, [args.slots])
        run = res["runs"][args.slots]
        out["serving"] = {"requests_per_s": run["requests_per_s"], "p50_s": run["p50_s"], "p99_s": run["p99_s"],
                          "mean_s": run["mean_s"], "slots": args.slots, "requests": args.requests,
                          "median_edges": res["median_edges"], "workload": res["workload"]}
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(h, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
