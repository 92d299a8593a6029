#!/usr/bin/env python3
"""Benchmark of the km1 label-propagation refinement core on one MI355X.

Workload (the sparse-matrix refinement case): the row-net hypergraph of a
seeded random 1,000,000 x 1,000,000 sparse matrix (about 10M pins, lognormal
row lengths, 70% banded columns), vertex weight = column degree, refined from
a random balanced start at k = 8 and at k = 64, eps = 0.03, 10 synchronous LP
rounds each.

One step is one pass of the whole hot path on resident device inputs: load
(incidence CSR + checks), and for each k: pin counts, 10 LP rounds (select /
approve / apply / finalize), all k-way gains, km1.  The reported value counts
the nominal pins of every LP round: 2 x 10 x P pins per step, divided by the
step time (so load, pin counts, gains and km1 are inside the time but add no
pins).

Also reported: per-round latency p50/p99 (each round timed alone with HIP
events), the recorded-hipGraph refine time, the select kernel's algorithmic
bandwidth against the 8 TB/s HBM peak (timed live with HIP events on the
kernel's stream during the timed steps), and the CPU oracle on a bounded
sample of the same workload.

usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "pins/s per LP refinement round (km1 gains), plain vs batched/served; p50/p99"
HBM_PEAK_GBS = 8000.0
KS = (8, 64)
ROUNDS = 10


def select_bytes(st, n, k):
    """Algorithmic bytes of one select launch: eligible bits n/8, 16 B per
    active vertex (part, offsets, weight), (12 + w_Lambda) B per active
    incidence (net id, w(e), the pin-count/singleton word of the own block,
    the Lambda bitset of ceil(k/32) words), 16 B per candidate written."""
    w_lambda = 4 * ((k + 31) // 32)
    return (n / 8.0 + 16.0 * st["boundary"] + (12.0 + w_lambda) * st["active_pins"] +
            16.0 * st["candidates"])


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    i = min(len(xs) - 1, max(0, int(round(q / 100.0 * (len(xs) - 1)))))
    return xs[i]


def cpu_baseline(inst, rounds_per_k):
    """Oracle (single-threaded C) on a bounded sample: `rounds_per_k` LP rounds
    at each k of the same workload, timed on this host."""
    from oracle import oracle as O
    h = O.Hypergraph(inst.n, inst.eptr, inst.pins, inst.c, inst.w)
    h.incidence()
    import numpy as np
    import synth
    pins_rounds = 0
    t_total = 0.0
    for k in KS:
        ik = synth.with_k(inst, k)
        L = O.lmax(O.total_vertex_weight(h), k, inst.eps)
        part = ik.part.copy()
        elig = np.ones(inst.n, np.uint8)
        for _ in range(rounds_per_k):
            t0 = time.perf_counter()
            part, elig, _, _ = O.lp_round(h, k, L, part, elig)
            t_total += time.perf_counter() - t0
            pins_rounds += inst.P
    return {"value": pins_rounds / t_total, "unit": "pins/s", "cores": 1, "kind": "oracle",
            "sample": "first %d LP rounds at k=%s of the same 1M x 1M instance (%d pins), "
                      "single-threaded C oracle, %.1f s" % (rounds_per_k, "/".join(map(str, KS)),
                                                           inst.P, t_total)}


BATCH_COUNT = 512
BATCH_ROUNDS = 8


def _events(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def batched_cpu_baseline(insts, budget_s):
    """Oracle on a bounded sample of the batch: members in order, every LP
    round of each, until about `budget_s` seconds of oracle time."""
    from oracle import oracle as O
    import numpy as np
    t_total, pin_rounds, done = 0.0, 0, 0
    for inst in insts:
        h = O.Hypergraph(inst.n, inst.eptr, inst.pins, inst.c, inst.w)
        h.incidence()
        L = O.lmax(O.total_vertex_weight(h), inst.k, inst.eps)
        part = inst.part.copy()
        elig = np.ones(inst.n, np.uint8)
        for _ in range(inst.rounds):
            t0 = time.perf_counter()
            part, elig, _, _ = O.lp_round(h, inst.k, L, part, elig)
            t_total += time.perf_counter() - t0
            pin_rounds += inst.P
        done += 1
        if t_total >= budget_s:
            break
    return {"value": pin_rounds / t_total, "unit": "pins/s", "cores": 1, "kind": "oracle",
            "sample": "all %d rounds of the first %d of the %d batch members (%d pin-rounds), "
                      "single-threaded C oracle, %.1f s" % (insts[0].rounds, done, len(insts),
                                                           pin_rounds, t_total)}


def batched_leg(args, H, dev):
    """The batched workload: 512 power-law hypergraphs (n log-uniform in
    [1e3, 5e5], k in {2,4,8,32,128}), 8 LP rounds each, refined by one
    recorded hipGraph launch over one segmented allocation, against the same
    512 refinements as sequential hg_refine calls (each a recorded graph)."""
    import torch
    import synth
    from paper_2010_10272_amd import segmented
    print("batched: generating %d instances ..." % args.batch_count, file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    insts = synth.batch_instances(seed=4, count=args.batch_count, rounds=BATCH_ROUNDS,
                                  workers=8)
    gen_s = time.perf_counter() - t0
    R = BATCH_ROUNDS
    P_total = sum(x.P for x in insts)
    members, ar = segmented.load_batch(insts, dev, rounds=R)
    part0 = ar.part_bytes.clone()
    torch.cuda.synchronize()
    print("batched: loaded (%.2f GB arena), sequential reference ..." % (ar.nbytes / 1e9),
          file=sys.stderr, flush=True)

    def timed(run, reps):
        xs = []
        for _ in range(reps):
            ar.part_bytes.copy_(part0)
            a, b = _events(torch)
            a.record()
            run()
            b.record()
            b.synchronize()
            xs.append(a.elapsed_time(b))
        return xs

    def snapshot():
        return (ar.part_bytes.clone(), torch.cat([mb.stats for mb in members]),
                torch.cat([mb.st.km1 for mb in members]))

    def seq():
        for mb in members:
            H.hg_refine(mb.g, mb.st, mb.eps, R, mb.stats, use_graph=True)

    timed(seq, 1)                                     # records every member's graph
    want = snapshot()
    seq_ms = timed(seq, args.batch_reps)

    b = H.hg_batch_create(members)
    default_sched = H.hg_batch_get_schedule(b)

    def bat():
        H.hg_batch_refine(b, R, use_graph=True)

    timed(bat, 1)                                     # records the batch graph
    got = snapshot()
    assert all(torch.equal(x, y) for x, y in zip(got, want)), "batched != sequential"
    default_ms = timed(bat, args.batch_reps)
    print("batched: autotuning ...", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    tuned = H.hg_batch_autotune(b, repeats=2)
    tune_s = time.perf_counter() - t0
    timed(bat, 1)
    got = snapshot()
    assert all(torch.equal(x, y) for x, y in zip(got, want)), "tuned batch != sequential"
    tuned_ms = timed(bat, args.batch_reps)
    # each batched round alone
    lat = []
    for _ in range(max(1, args.batch_reps // 2)):
        ar.part_bytes.copy_(part0)
        H.hg_batch_start(b)
        for r in range(R):
            a, e = _events(torch)
            a.record()
            H.hg_batch_round(b, r)
            e.record()
            e.synchronize()
            lat.append(a.elapsed_time(e))
    stats = [H.stats_to_dicts(mb.stats) for mb in members]
    b.free()
    best_ms = min(percentile(default_ms, 50), percentile(tuned_ms, 50))
    out = {
        "metric": "pins/s per LP round, batched",
        "value": P_total * R / (best_ms / 1e3),
        "unit": "pins/s",
        "members": len(insts),
        "rounds": R,
        "P_total": P_total,
        "n_total": sum(x.n for x in insts),
        "batch_ms": best_ms,
        "batch_ms_default_schedule": percentile(default_ms, 50),
        "batch_ms_tuned_schedule": percentile(tuned_ms, 50),
        "sequential_ms": percentile(seq_ms, 50),
        "sequential_value": P_total * R / (percentile(seq_ms, 50) / 1e3),
        "speedup_vs_sequential": percentile(seq_ms, 50) / best_ms,
        "round_latency": {"p50_ms": percentile(lat, 50), "p99_ms": percentile(lat, 99)},
        "schedule_default": default_sched,
        "schedule_tuned": tuned,
        "tune_s": tune_s,
        "moves_total": sum(s["approved"] for st in stats for s in st),
        "active_pins_total": sum(s["active_pins"] for st in stats for s in st),
        "generate_s": gen_s,
        "arena_bytes": ar.nbytes,
        "check": "final partitions, round records and km1 of all members identical to "
                 "512 sequential hg_refine calls",
    }
    if not args.no_cpu:
        out["cpu_baseline"] = batched_cpu_baseline(insts, args.batch_cpu_s)
    for mb in members:
        mb.g.free()
    del members, ar
    torch.cuda.empty_cache()
    return out


def plain_leg(args, H, dev):
    """The plain workload (module docstring): returns the JSON record."""
    import torch
    import synth
    print("generating workload ...", file=sys.stderr, flush=True)
    inst = synth.sparse_matrix(KS[0])
    n, m, P = inst.n, inst.m, inst.P
    parts = {k: torch.as_tensor(synth.with_k(inst, k).part).to(dev) for k in KS}
    eptr = torch.as_tensor(inst.eptr).to(dev)
    pins = torch.as_tensor(inst.pins).to(dev)
    c = torch.as_tensor(inst.c).to(dev)
    w = torch.as_tensor(inst.w).to(dev)
    kmax = max(KS)
    ws_bytes = H.hg_workspace_size(n, m, P, kmax)
    bufs = (torch.empty(n + 1, dtype=torch.int64, device=dev),
            torch.empty(P, dtype=torch.int32, device=dev),
            torch.empty(ws_bytes, dtype=torch.uint8, device=dev))
    g0 = H.hg_load_csr(n, eptr, pins, c, w, k_max=kmax, device=dev, out=bufs)
    states = {k: H.State(g0, k, parts[k]) for k in KS}
    g0.free()
    stats = {k: torch.zeros(ROUNDS * H.STATS_WORDS, dtype=torch.int64, device=dev) for k in KS}
    gains = torch.empty(n * kmax, dtype=torch.int64, device=dev)
    km1_out = torch.empty(1, dtype=torch.int64, device=dev)

    phase_ms = {p: 0.0 for p in H.HG_PHASES}
    timed_rounds = [0]

    def step(collect):
        g = H.hg_load_csr(n, eptr, pins, c, w, k_max=kmax, device=dev, out=bufs)
        H.hg_timing_enable(g, True)
        for k in KS:
            st = states[k]
            st.part.copy_(parts[k])
            H.hg_refine(g, st, inst.eps, ROUNDS, stats[k], use_graph=False)
            H.hg_gains(g, k, st.part, st.netstate, gains=gains[:n * k])
            H.hg_km1(g, k, st.netstate, out=km1_out)
        ms, r = H.hg_timing_collect(g)     # waits for the step's last round
        if collect:
            for p in ms:
                phase_ms[p] += ms[p]
            timed_rounds[0] += r
        g.free()

    print("warmup ...", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    print("timing %d steps ..." % args.steps, file=sys.stderr, flush=True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        step(True)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = e0.elapsed_time(e1)
    elapsed = max(wall, gpu_ms / 1e3)
    ms_per_step = elapsed * 1e3 / args.steps
    value = len(KS) * ROUNDS * P * args.steps / elapsed

    per_k = {k: H.stats_to_dicts(stats[k]) for k in KS}
    for k in KS:
        for s in per_k[k]:
            assert s["km1_delta"] == s["km1_delta_recomputed"], "attributed km1 mismatch"
    sel_bytes_step = sum(select_bytes(s, n, k) for k in KS for s in per_k[k])
    sel_launches_step = len(KS) * ROUNDS
    sel_ms_avg = phase_ms["select"] / max(1, timed_rounds[0])
    achieved = (sel_bytes_step / sel_launches_step) / (sel_ms_avg / 1e3) / 1e9

    # per-round latency: each round timed alone (events around hg_lp_round)
    lat = {}
    g = H.hg_load_csr(n, eptr, pins, c, w, k_max=kmax, device=dev, out=bufs)
    one = torch.zeros(H.STATS_WORDS, dtype=torch.int64, device=dev)
    for k in KS:
        st = states[k]
        L = H.hg_max_block_weight(g, k, inst.eps)
        xs = []
        for _ in range(args.latency_reps):
            st.part.copy_(parts[k])
            H.hg_compute_pincounts(g, st)
            st.eligible.fill_(1)
            for r in range(ROUNDS):
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record()
                H.hg_lp_round(g, st, L, one, moved=False)
                b.record()
                b.synchronize()
                xs.append(a.elapsed_time(b))
        lat["k%d" % k] = {"p50_ms": percentile(xs, 50), "p99_ms": percentile(xs, 99)}
    # recorded hipGraph replay of the same refinement
    graph_ms = {}
    for k in KS:
        st = states[k]
        xs = []
        for _ in range(args.latency_reps + 1):
            st.part.copy_(parts[k])
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            H.hg_refine(g, st, inst.eps, ROUNDS, stats[k], use_graph=True)
            b.record()
            b.synchronize()
            xs.append(a.elapsed_time(b))
        graph_ms["k%d" % k] = percentile(xs[1:], 50)       # first call records the graph
        assert H.stats_to_dicts(stats[k]) == per_k[k], "graph replay differs"
    g.free()

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "pins/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {
            "workload": "sparse-matrix row-net hypergraph 1M x 1M (%d pins), k=8 and k=64, "
                        "eps=0.03, 10 synchronous LP rounds per k; one step = load + "
                        "(pin counts + 10 rounds + gains + km1) per k" % P,
            "n": n, "m": m, "P": P, "k": list(KS), "rounds": ROUNDS, "eps": inst.eps,
            "seed": 2, "parallelism": "single GPU",
        },
        "roofline": {
            "kernel": "k_select_light (LP select sweep)",
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "avg_launch_us": sel_ms_avg * 1e3,
            "alg_bytes_per_launch": sel_bytes_step / sel_launches_step,
        },
        "phase_ms_per_round": {p: phase_ms[p] / max(1, timed_rounds[0]) for p in phase_ms},
        "round_latency": lat,
        "graph_refine_ms": graph_ms,
        "km1_final": {"k%d" % k: per_k[k][-1]["km1_after"] for k in KS},
    }
    if args.calibrate_copy > 0:
        nb = args.calibrate_copy << 20
        src = torch.ones(nb // 4, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["calibrate_copy_bytes"] = nb
        del src, dst
    if not args.no_cpu:
        print("cpu baseline ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(inst, args.cpu_rounds)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-rounds", type=int, default=4)
    ap.add_argument("--latency-reps", type=int, default=5)
    ap.add_argument("--legs", default="plain,batched",
                    help="comma list of plain, batched")
    ap.add_argument("--batch-count", type=int, default=BATCH_COUNT)
    ap.add_argument("--batch-reps", type=int, default=5)
    ap.add_argument("--batch-cpu-s", type=float, default=8.0)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="also run one plain device-to-device copy of MIB MiB (a known "
                         "byte count for scaling HBM traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2010_10272_amd import hgref as H

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    legs = set(args.legs.split(","))
    out = plain_leg(args, H, dev) if "plain" in legs else {"metric": METRIC}
    if "batched" in legs:
        torch.cuda.empty_cache()
        out["batched"] = batched_leg(args, H, dev)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
