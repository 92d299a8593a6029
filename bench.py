#!/usr/bin/env python3
"""Benchmark of the km1 label-propagation refinement core on one MI355X.

Headline workload (the largest plain single-GPU case): a seeded VLSI-like
netlist, 4,000,000 cells on a 2000 x 2000 grid, 4,200,000 nets (sizes 2-5
with probability 0.9, else 6-200; 99% inside a 16 x 16 window, 1% global),
about 56.5M pins, cell weights U{1..8}, refined from a horizontal-strip start
at k = 16, eps = 0.03, 10 synchronous LP rounds.

One step is one pass of the whole hot path on resident device inputs: load
(incidence CSR + checks), pin counts, 10 LP rounds (select / approve / apply
/ finalize), all k-way gains, km1.  The reported value counts the nominal
pins of every LP round, 10 x P pins per step, divided by the step time (load,
pin counts, gains and km1 are inside the time but add no pins).

Beside it, the same measurement on the sparse-matrix workload (1M x 1M row-net
matrix, about 10M pins, k = 8 and 64) and on the tiny instance (n = m =
10,000, k = 2, 5 rounds), then the batched, served, monotone, gain-cache,
rebalancing and contraction legs.  For each plain workload: the select
kernel's and the whole round's algorithmic bandwidth against the 8 TB/s HBM
peak (round records over the library's per-phase HIP events, recorded on the
kernels' stream during the last timed step), per-round latency p50/p99, the
recorded-hipGraph refine time, and the CPU oracle on a bounded sample of the
same rounds, whose records and partitions must equal the timed run's.

usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--legs ...]
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


def _w_lambda(k):
    return 4 * ((k + 31) // 32)


def select_bytes(st, n, k):
    """Algorithmic bytes of one select launch: eligible bits n/8, 16 B per
    active vertex (part, offsets, weight), (12 + w_Lambda) B per active
    incidence (net id, w(e), the pin-count/singleton word of the own block,
    the Lambda bitset of ceil(k/32) words), 16 B per candidate written."""
    return (n / 8.0 + 16.0 * st["boundary"] + (12.0 + _w_lambda(k)) * st["active_pins"] +
            16.0 * st["candidates"])


def approve_bytes(st, n, k):
    """Approval and apply of one round: 32 B per candidate (its word read by
    the tile sums and the approval, its weight), 4 B per approved move, and
    the apply: 16 B per mover (part, offsets, weight, flag), 20 B per moved
    incidence (net id, two Phi read-modify-writes)."""
    return 32.0 * st["candidates"] + 20.0 * st["approved"] + 20.0 * st["moved_pins"]


def finalize_bytes(st, n, k):
    """Finalize of one round: 8 B per touched net (offsets, flag, record),
    4 B per pin of a touched net (the pin ids whose eligibility is set), the
    next eligible set n/8."""
    return 8.0 * st["touched_nets"] + 4.0 * st["touched_pins"] + n / 8.0


PHASE_BYTES = {"select": select_bytes, "approve": approve_bytes, "finalize": finalize_bytes}


def roofline_of(name, alg_bytes, ms):
    """A roofline record: algorithmic bytes of one call over its time."""
    achieved = alg_bytes / (ms / 1e3) / 1e9
    return {"kernel": name, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "alg_bytes": alg_bytes, "ms": ms}


def timed_oracle(fn):
    """Seconds one oracle call takes on this host (one thread)."""
    t0 = time.perf_counter()
    out = fn()
    return time.perf_counter() - t0, out


def host_info():
    """The host the oracle baseline ran on: CPU model, logical CPUs (all and
    usable by this process), the oracle's compiler and flags."""
    import subprocess
    from oracle import oracle as O
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        cc = subprocess.run([O.CC, "--version"], capture_output=True, text=True,
                            timeout=10).stdout.splitlines()[0]
    except (OSError, IndexError, subprocess.SubprocessError):
        cc = None
    return {"cpu_model": model, "nproc": os.cpu_count(),
            "usable_cpus": len(os.sched_getaffinity(0)), "compiler": cc,
            "flags": " ".join(O.CFLAGS), "threads_used": 1}


PROFILES = os.path.join(ROOT, "profiles")


def measured_traffic(profile, prefix):
    """HBM-side bytes per launch of one kernel from a committed rocprofv3
    counter summary, or None when that kernel's sources changed since the
    counters were taken (their SHA-256 is recorded with them)."""
    import hashlib
    import re
    try:
        text = open(os.path.join(PROFILES, profile)).read()
    except OSError:
        return None
    got = dict(re.findall(r"^(%s_[a-z_0-9]+): (.+)$" % prefix, text, re.M))
    key = prefix + "_traffic_bytes_per_launch"
    if key not in got:
        return None
    h = hashlib.sha256()
    for rel in got[prefix + "_sources"].split():
        try:
            h.update(open(os.path.join(ROOT, rel), "rb").read())
        except OSError:
            return None
    if h.hexdigest() != got.get(prefix + "_sources_sha256", "").strip():
        return None
    return float(got[key])


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    i = min(len(xs) - 1, max(0, int(round(q / 100.0 * (len(xs) - 1)))))
    return xs[i]


BATCH_COUNT = 512
BATCH_ROUNDS = 8


def _events(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def batched_cpu_baseline(insts, budget_s, members, H):
    """Oracle on a bounded sample of the batch: members in order, every LP
    round of each, until about `budget_s` seconds of oracle time; each
    sampled member's round records and final partition must equal the
    batched run's."""
    from oracle import oracle as O
    import numpy as np
    t_total, pin_rounds, done = 0.0, 0, 0
    for inst, mb in zip(insts, members):
        h = O.Hypergraph(inst.n, inst.eptr, inst.pins, inst.c, inst.w)
        h.incidence()
        L = O.lmax(O.total_vertex_weight(h), inst.k, inst.eps)
        part = inst.part.copy()
        elig = np.ones(inst.n, np.uint8)
        recs = []
        for _ in range(inst.rounds):
            t0 = time.perf_counter()
            part, elig, _, st = O.lp_round(h, inst.k, L, part, elig)
            t_total += time.perf_counter() - t0
            pin_rounds += inst.P
            recs.append(st)
        got = H.stats_to_dicts(mb.stats)
        for r, want in enumerate(recs):
            got[r].pop("km1_delta_recomputed")
            assert got[r] == want, "batch member %d round %d differs from the oracle" % (done, r)
        assert np.array_equal(mb.st.part.cpu().numpy(), part), "batch member %d differs" % done
        done += 1
        if t_total >= budget_s:
            break
    return {"value": pin_rounds / t_total, "unit": "pins/s", "cores": 1, "kind": "oracle",
            "host": host_info(),
            "sample": "all %d rounds of the first %d of the %d batch members (%d pin-rounds), "
                      "single-threaded C oracle, %.1f s; their records and partitions equal "
                      "the batched run's" % (insts[0].rounds, done, len(insts),
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
        out["cpu_baseline"] = batched_cpu_baseline(insts, args.batch_cpu_s, members, H)
    for mb in members:
        mb.g.free()
    del members, ar
    torch.cuda.empty_cache()
    return out


SERVED_RATE = 200.0
SERVED_BUDGET = 16 << 30      # job memory of the server (admission binds under bursts)
SERVED_TABLE = 64 << 20
SERVED_BIG_PINS = 8_000_000   # jobs this large (the grid netlists) take the server's second lane


def _sleep_until(clock, due_ms):
    while True:
        left = due_ms - clock()
        if left <= 0:
            return
        time.sleep(left / 1e3 if left > 1.0 else 0)


def _lat_summary(lat_ms, pin_rounds, t_first, t_last):
    span = (t_last - t_first) / 1e3
    return {"requests": len(lat_ms), "p50_ms": percentile(lat_ms, 50),
            "p99_ms": percentile(lat_ms, 99), "max_ms": max(lat_ms) if lat_ms else None,
            "mean_ms": sum(lat_ms) / max(1, len(lat_ms)), "makespan_s": span,
            "value": pin_rounds / span if span > 0 else None, "unit": "pins/s"}


def served_leg(args, H, dev):
    """The served workload: an open-loop Poisson trace (200 requests/s; 95%
    hypergraphs of the batched size distribution, 5% 2M-cell grid netlists;
    k in {2,4,8,32,128}; 10 rounds each) against the request server (16 GB of
    job memory) and against the plain one-at-a-time path (load, hg_refine,
    copy back, per request in arrival order).  Latency = completion minus
    scheduled arrival.  Then the same requests all at once (a burst) for the
    throughput each path sustains.  Every served result is checked against the
    plain path's."""
    import numpy as np
    import torch
    import synth
    print("served: generating the request pool ...", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    trace = synth.served_trace(seed=5, rate=SERVED_RATE, seconds=args.served_seconds)
    small, big = synth.served_pool(seed=5, workers=8)
    gen_s = time.perf_counter() - t0

    def pinned(a, dt):
        return torch.from_numpy(np.ascontiguousarray(a)).to(dt).pin_memory()

    hosts = {}

    def host_of(req):
        key = (req.big, req.pool)
        if key not in hosts:
            inst = (big if req.big else small)[req.pool]
            unit_c = bool(np.all(inst.c == 1))
            unit_w = bool(np.all(inst.w == 1))
            hosts[key] = {"inst": inst, "eptr": pinned(inst.eptr, torch.int64),
                          "pins": pinned(inst.pins, torch.int32),
                          "vwgt": None if unit_c else pinned(inst.c, torch.int32),
                          "ewgt": None if unit_w else pinned(inst.w, torch.int32), "parts": {}}
        h = hosts[key]
        if req.k not in h["parts"]:
            h["parts"][req.k] = pinned(synth.with_k(h["inst"], req.k).part, torch.int32)
        return h

    reqs = [(r, host_of(r)) for r in trace]
    # every request's results in three page-locked slabs (one allocation each
    # instead of three per request), cleared before each run
    n_off = np.cumsum([0] + [h["inst"].n for r, h in reqs])
    s_off = np.cumsum([0] + [r.rounds * H.STATS_WORDS for r, h in reqs])
    slab = (torch.zeros(int(n_off[-1]), dtype=torch.int32, pin_memory=True),
            torch.zeros(int(s_off[-1]), dtype=torch.int64, pin_memory=True),
            torch.zeros(len(reqs), dtype=torch.int64, pin_memory=True))

    def outputs_all():
        for x in slab:
            x.zero_()
        return [(slab[0][n_off[i]:n_off[i + 1]], slab[1][s_off[i]:s_off[i + 1]],
                 slab[2][i:i + 1]) for i in range(len(reqs))]

    pin_rounds = sum(h["inst"].P * r.rounds for r, h in reqs)
    print("served: %d requests (%d big), %.2e pin-rounds" % (
        len(reqs), sum(r.big for r in trace), pin_rounds), file=sys.stderr, flush=True)

    def run_served(burst):
        outs = outputs_all()
        srv = H.hg_server_create(SERVED_BUDGET + SERVED_TABLE, table_bytes=SERVED_TABLE,
                                 max_active=256, device=dev, big_pins=SERVED_BIG_PINS)
        clock = lambda: H.hg_server_now_ms(srv)          # noqa: E731
        start = clock() + 20.0
        ids = []
        for (r, h), out in zip(reqs, outs):
            due = start if burst else start + r.arrival_s * 1e3
            if not burst:
                _sleep_until(clock, due)
            inst = h["inst"]
            ids.append(H.hg_server_submit(srv, inst.n, h["eptr"], h["pins"], h["parts"][r.k],
                                          r.k, r.rounds, r.eps, vwgt=h["vwgt"], ewgt=h["ewgt"],
                                          arrival_ms=due, results=out))
        left = H.hg_server_drain(srv, max(120.0, 6 * args.served_seconds) * 1e3)
        assert left == 0, "server did not finish"
        infos = [H.hg_server_info(srv, i) for i in ids]
        assert all(x["status"] == H.HG_OK for x in infos), "a served request failed"
        lat = [x["done_ms"] - x["arrival_ms"] for x in infos]
        res = _lat_summary(lat, pin_rounds, start, max(x["done_ms"] for x in infos))
        res["server"] = H.hg_server_get_stats(srv)
        small = [x for (r, h), x in zip(reqs, infos) if not r.big]
        res["small_p50_parts_ms"] = {
            "queued": percentile([x["admit_ms"] - x["arrival_ms"] for x in small], 50),
            "load": percentile([x["loaded_ms"] - x["admit_ms"] for x in small], 50),
            "rounds_and_copy": percentile([x["done_ms"] - x["loaded_ms"] for x in small], 50)}
        srv.free()
        return res, outs

    def run_plain(burst):
        outs = outputs_all()
        clock = lambda: time.perf_counter() * 1e3        # noqa: E731
        start = clock() + 20.0
        lat, t_last = [], start
        parts = {"queued": [], "load": [], "rounds_and_copy": []}
        stats = torch.zeros(16 * H.STATS_WORDS, dtype=torch.int64, device=dev)
        for (r, h), out in zip(reqs, outs):
            due = start if burst else start + r.arrival_s * 1e3
            if not burst:
                _sleep_until(clock, due)
            inst = h["inst"]
            t_begin = clock()
            g = H.hg_load_csr(inst.n, h["eptr"], h["pins"], h["vwgt"], h["ewgt"], k_max=r.k,
                              device=dev)
            t_loaded = clock()
            st = H.State(g, r.k, h["parts"][r.k])
            H.hg_refine(g, st, r.eps, r.rounds, stats, use_graph=False)
            out[0].copy_(st.part, non_blocking=True)
            out[1].copy_(stats[:r.rounds * H.STATS_WORDS], non_blocking=True)
            out[2].copy_(st.km1, non_blocking=True)
            torch.cuda.synchronize()
            t_last = clock()
            lat.append(t_last - due)
            if not r.big:
                parts["queued"].append(t_begin - due)
                parts["load"].append(t_loaded - t_begin)
                parts["rounds_and_copy"].append(t_last - t_loaded)
            g.free()
        res = _lat_summary(lat, pin_rounds, start, t_last)
        res["small_p50_parts_ms"] = {x: percentile(v, 50) for x, v in parts.items()}
        return res, outs

    res = {"rate_per_s": SERVED_RATE, "seconds": args.served_seconds, "requests": len(reqs),
           "big_requests": sum(r.big for r in trace), "pin_rounds": pin_rounds,
           "job_memory_bytes": SERVED_BUDGET, "generate_s": gen_s,
           "pool": {"small": len(small), "big": len(big)}}
    for mode in ("open_loop", "burst"):
        burst = mode == "burst"
        print("served: %s, server ..." % mode, file=sys.stderr, flush=True)
        srv_res, _ = run_served(burst)
        served = [x.numpy().copy() for x in slab]
        print("served: %s, plain one-at-a-time ..." % mode, file=sys.stderr, flush=True)
        pl_res, _ = run_plain(burst)
        assert np.array_equal(served[0], slab[0].numpy()), "served partition differs from plain"
        assert np.array_equal(served[1], slab[1].numpy()), "served round records differ"
        assert np.array_equal(served[2], slab[2].numpy()), "served km1 differs"
        del served
        res[mode] = {"served": srv_res, "plain": pl_res}
    res["check"] = ("every served request's partition, round records and km1 identical to the "
                    "plain one-at-a-time path, in both modes")
    return res


_SPARSE = {}


def sparse_instance():
    """The sparse-matrix workload (generated once per run)."""
    import synth
    if "inst" not in _SPARSE:
        _SPARSE["inst"] = synth.sparse_matrix(KS[0])
    return _SPARSE["inst"]


def monotone_leg(args, H, dev):
    """Monotone rounds (exact gains of each round's approved moves in (gain
    desc, id asc) order, best prefix applied) on the sparse-matrix workload at
    k = 8 and 64, 10 rounds, beside plain rounds on the same start; and the
    exact gains of a 100,000-move sequence on their own."""
    import numpy as np
    import torch
    import synth
    inst = sparse_instance()
    out = {}
    for k in KS:
        ik = synth.with_k(inst, k)
        g = H.hg_load_csr(inst.n, inst.eptr, inst.pins, inst.c, inst.w, k_max=k, device=dev)
        st = H.State(g, k, ik.part)
        ws = H.moves_workspace(g, k)
        stats = torch.zeros(ROUNDS * H.STATS_WORDS, dtype=torch.int64, device=dev)
        part0 = st.part.clone()
        res = {}
        for mode in ("plain", "monotone"):
            xs = []
            for rep in range(args.mono_reps + 1):
                st.part.copy_(part0)
                a, b = _events(torch)
                a.record()
                if mode == "plain":
                    H.hg_refine(g, st, inst.eps, ROUNDS, stats, use_graph=False)
                else:
                    H.hg_refine_exact(g, st, inst.eps, ROUNDS, stats, ws)
                b.record()
                b.synchronize()
                if rep:
                    xs.append(a.elapsed_time(b))
            recs = H.stats_to_dicts(stats)
            kms = [r["km1_after"] for r in recs]
            res[mode] = {"refine_ms": percentile(xs, 50), "round_ms": percentile(xs, 50) / ROUNDS,
                         "km1_after_rounds": kms, "moves": sum(r["approved"] for r in recs),
                         "pins_per_s": inst.P * ROUNDS / (percentile(xs, 50) / 1e3)}
            if mode == "monotone":
                assert all(b <= a for a, b in zip(kms, kms[1:])), "monotone km1 increased"
        # exact gains of one explicit sequence: 100,000 random moves
        rng = np.random.default_rng(9)
        t = min(100_000, inst.n)
        mu = torch.as_tensor(rng.permutation(inst.n)[:t].astype(np.int32), device=dev)
        mt = ((part0[mu.long()] + 1 + torch.as_tensor(rng.integers(0, k - 1, t), device=dev))
              % k).to(torch.int32)
        st.part.copy_(part0)
        H.hg_compute_pincounts(g, st)
        gains = torch.empty(t, dtype=torch.int64, device=dev)
        xs = []
        for rep in range(args.mono_reps + 1):
            a, b = _events(torch)
            a.record()
            H.hg_move_gains(g, k, st.part, st.phi, mu, mt, ws, gains=gains)
            b.record()
            b.synchronize()
            if rep:
                xs.append(a.elapsed_time(b))
        deg = (g.vptr[1:] - g.vptr[:-1])[mu.long()].sum().item()
        mg_ms = percentile(xs, 50)
        res["move_gains"] = {"moves": t, "incidences": int(deg), "ms": mg_ms,
                             "incidences_per_s": deg / (mg_ms / 1e3),
                             # per incidence: net id read by the three passes (12 B),
                             # the (e, a) and (e, b) cells cleared (24 B) and updated
                             # (24 B), then Phi and the cells read (36 B) plus w(e) (4 B);
                             # per move: the move (8 B), offsets (16 B), part (4 B), gain
                             "roofline": roofline_of("k_seq_init + k_seq_collect + k_seq_gains",
                                                     100.0 * deg + 36.0 * t, mg_ms)}
        if not args.no_cpu:
            from oracle import oracle as O
            h = O.Hypergraph(inst.n, inst.eptr, inst.pins, inst.c, inst.w)
            h.incidence()
            dt, want = timed_oracle(lambda: O.move_gains(h, k, ik.part, mu.cpu().numpy(),
                                                         mt.cpu().numpy()))
            assert np.array_equal(want, gains.cpu().numpy()), "move gains differ from the oracle"
            res["move_gains"]["cpu_baseline"] = {
                "value": deg / dt, "unit": "incidences/s", "cores": 1, "kind": "oracle",
                "host": host_info(),
                "sample": "the same %d-move sequence, once" % t}
        out["k%d" % k] = res
        g.free()
    return out


def cached_leg(args, H, dev):
    """Gain-cache rounds (select reads b, w(I) and the penalty rows; the
    finalize applies the round's net deltas) beside plain rounds on the
    sparse-matrix workload at k = 8 and 64, 10 rounds from the same start;
    both must give the same partition and round records.  Per-phase times
    come from the library's own event timing."""
    import numpy as np
    import torch
    import synth
    inst = sparse_instance()
    out = {}
    for k in KS:
        ik = synth.with_k(inst, k)
        g = H.hg_load_csr(inst.n, inst.eptr, inst.pins, inst.c, inst.w, k_max=k, device=dev)
        st = H.State(g, k, ik.part)
        cache = H.gain_cache(g, k)
        stats = torch.zeros(ROUNDS * H.STATS_WORDS, dtype=torch.int64, device=dev)
        part0 = st.part.clone()
        res, finals = {}, {}
        for mode in ("plain", "cached"):
            xs = []
            phases = {p: 0.0 for p in H.HG_PHASES}
            timed = 0
            for rep in range(args.mono_reps + 2):
                st.part.copy_(part0)
                profile = rep == args.mono_reps + 1
                H.hg_timing_enable(g, profile)
                a, b = _events(torch)
                a.record()
                if mode == "plain":
                    H.hg_refine(g, st, inst.eps, ROUNDS, stats, use_graph=False)
                else:
                    H.hg_refine_cached(g, st, inst.eps, ROUNDS, stats, cache)
                b.record()
                b.synchronize()
                if profile:
                    ph, timed = H.hg_timing_collect(g)
                    phases = {p: v / max(timed, 1) for p, v in ph.items()}
                    H.hg_timing_enable(g, False)
                elif rep:
                    xs.append(a.elapsed_time(b))
            finals[mode] = (st.part.clone(), stats.clone())
            res[mode] = {"refine_ms": percentile(xs, 50),
                         "round_ms": percentile(xs, 50) / ROUNDS,
                         "phase_ms_per_round": phases,
                         "pins_per_s": inst.P * ROUNDS / (percentile(xs, 50) / 1e3)}
        assert torch.equal(finals["plain"][0], finals["cached"][0]), "cached rounds differ"
        assert torch.equal(finals["plain"][1], finals["cached"][1]), "cached records differ"
        res["cache_bytes"] = cache.numel() * 4
        # the cached select per launch: eligible and moved flags (2n), candidate
        # words (8n), and per eligible vertex part, b, w(I) and its padded row
        recs = H.stats_to_dicts(finals["cached"][1])
        ks = (k + 3) // 4 * 4
        sel_bytes = sum(10.0 * inst.n + r["eligible"] * (12.0 + 4.0 * ks) + 16.0 * r["candidates"]
                        for r in recs) / len(recs)
        res["roofline"] = roofline_of("k_select_cached", sel_bytes,
                                      res["cached"]["phase_ms_per_round"]["select"])
        if not args.no_cpu:
            from oracle import oracle as O
            h = O.Hypergraph(inst.n, inst.eptr, inst.pins, inst.c, inst.w)
            L = H.hg_max_block_weight(g, k, inst.eps)
            dt, (p1, s1, _) = timed_oracle(lambda: O.refine(h, k, L, 1, ik.part))
            # one cached round from the same start must equal the oracle's round
            st.part.copy_(part0)
            one = torch.zeros(H.STATS_WORDS, dtype=torch.int64, device=dev)
            H.hg_refine_cached(g, st, inst.eps, 1, one, cache)
            got = H.stats_to_dicts(one)[0]
            got.pop("km1_delta_recomputed")
            assert got == s1[0], "cached round record differs from the oracle"
            assert np.array_equal(st.part.cpu().numpy(), p1), "cached round differs from oracle"
            res["cpu_baseline"] = {"value": inst.P / dt, "unit": "pins/s", "cores": 1,
                                   "kind": "oracle", "host": host_info(),
                                   "sample": "one label-propagation round, k = %d (equal to the "
                                             "GPU's cached round: partition and record)" % k}
        out["k%d" % k] = res
        g.free()
    return out


def rebalance_leg(args, H, dev):
    """Rebalancing rounds on the sparse-matrix workload at k = 8 and 64 from
    an overloaded start: a seeded 10% of the vertices piled into block 0 (and
    block 1 at k = 64) on top of the strip partition; 4 rounds."""
    import numpy as np
    import torch
    import synth
    inst = sparse_instance()
    out = {}
    RB_ROUNDS = 4
    for k in KS:
        ik = synth.with_k(inst, k)
        rng = np.random.default_rng(11)
        part0 = ik.part.copy()
        pick = rng.random(inst.n) < 0.1
        part0[pick] = rng.choice(np.array([0] if k == 8 else [0, 1], np.int32), int(pick.sum()))
        g = H.hg_load_csr(inst.n, inst.eptr, inst.pins, inst.c, inst.w, k_max=k, device=dev)
        L = H.hg_max_block_weight(g, k, inst.eps)
        st = H.State(g, k, part0)
        ws = H.rebalance_workspace(g, k)
        stats = torch.zeros(RB_ROUNDS * H.STATS_WORDS, dtype=torch.int64, device=dev)
        p0 = st.part.clone()
        xs = []
        for rep in range(args.mono_reps + 1):
            st.part.copy_(p0)
            st.eligible.zero_()
            H.hg_compute_pincounts(g, st)
            km0 = int(st.km1.item())
            w0 = int(st.block_w.max().item())
            a, b = _events(torch)
            a.record()
            H.hg_rebalance(g, st, L, RB_ROUNDS, stats, ws)
            b.record()
            b.synchronize()
            if rep:
                xs.append(a.elapsed_time(b))
        recs = H.stats_to_dicts(stats)
        ms = percentile(xs, 50)
        # per round, the terms every rebalancing round must move: the cache
        # rows of the considered vertices (filled from their incidences, then
        # read: (12 + w_Lambda) B per incidence, 2 x (8 + 4 ks) B per vertex),
        # flags / keys / candidate words of all vertices (2n + 8n + 8n), the
        # applied moves (16 B each, 20 B per incidence) and the finalize of the
        # touched nets (8 B each; their pins are left out, the records do not
        # count them, so this is a lower bound)
        w_l = 4 * ((k + 31) // 32)
        ks = (k + 3) // 4 * 4
        rb_bytes = sum((12.0 + w_l) * r["active_pins"] + 2 * (8.0 + 4 * ks) * r["eligible"] +
                       18.0 * inst.n + 16.0 * r["approved"] + 20.0 * r["moved_pins"] +
                       8.0 * r["touched_nets"] for r in recs)
        base = None
        if not args.no_cpu:
            from oracle import oracle as O
            h = O.Hypergraph(inst.n, inst.eptr, inst.pins, inst.c, inst.w)
            h.incidence()
            dt, (p1, e1, _, s1) = timed_oracle(lambda: O.rebalance_round(
                h, k, L, part0, np.zeros(inst.n, np.uint8)))
            # the first round from the same start, compared element by element
            st.part.copy_(p0)
            st.eligible.zero_()
            H.hg_compute_pincounts(g, st)
            one = torch.zeros(H.STATS_WORDS, dtype=torch.int64, device=dev)
            H.hg_rebalance(g, st, L, 1, one, ws)
            got = H.stats_to_dicts(one)[0]
            got.pop("km1_delta_recomputed")
            assert got == s1, "rebalancing record differs from the oracle"
            assert np.array_equal(st.part.cpu().numpy(), p1), "rebalancing differs from oracle"
            assert np.array_equal(st.eligible.cpu().numpy(), e1), "rebalancing eligible differs"
            base = {"value": inst.P / dt, "unit": "pins/s", "cores": 1, "kind": "oracle",
                    "host": host_info(),
                    "sample": "the first rebalancing round, k = %d (equal to the GPU's: "
                              "partition, eligible set and record)" % k}
        out["k%d" % k] = {"roofline": roofline_of("rebalancing round (all kernels)", rb_bytes,
                                                  ms),
                          "cpu_baseline": base,
            "rounds": RB_ROUNDS, "ms": ms, "round_ms": ms / RB_ROUNDS,
            "l_max": L, "max_block_weight_before": w0,
            "max_block_weight_after": [r["max_block_weight"] for r in recs],
            "moves": [r["approved"] for r in recs], "considered": recs[0]["eligible"],
            "km1_before": km0, "km1_after": recs[-1]["km1_after"],
            "pins_per_s": inst.P * RB_ROUNDS / (ms / 1e3)}
        g.free()
    return out


def contract_leg(args, H, dev):
    """Contraction of the sparse-matrix hypergraph under a seeded clustering
    of the shape one coarsening pass makes (synth.neighbour_clusters: half of
    the vertices join a neighbour): pins/s, the coarse sizes, and the time of
    the oracle's contraction of the same input on the host."""
    import torch
    import synth
    inst = sparse_instance()
    cl = synth.neighbour_clusters(inst)
    g = H.hg_load_csr(inst.n, inst.eptr, inst.pins, inst.c, inst.w, k_max=2, device=dev)
    out = H.Coarse(g)
    ws = H.contract_workspace(g)
    cl_d = torch.as_tensor(cl).to(dev)
    xs = []
    for rep in range(args.mono_reps + 2):
        a, b = _events(torch)
        a.record()
        H.hg_contract(g, cl_d, out, ws)
        b.record()
        b.synchronize()
        if rep:
            xs.append(a.elapsed_time(b))
    H.hg_sync_status(g)
    nc, mc, pc = out.read_sizes()
    ms = percentile(xs, 50)
    # what any contraction moves: cluster ids and map (4n + 4n), net offsets
    # (8m), pins read and mapped (4P + 4P), the coarse weights, offsets, pins
    # and net weights written (4n' + 8m' + 4P' + 4m')
    alg = 8.0 * inst.n + 8.0 * inst.m + 8.0 * inst.P + 4.0 * nc + 12.0 * mc + 4.0 * pc
    res = {"ms": ms, "pins_per_s": inst.P / (ms / 1e3), "n": inst.n, "m": inst.m, "P": inst.P,
           "coarse": {"n": nc, "m": mc, "P": pc}, "workspace_bytes": ws.numel(),
           "roofline": roofline_of("contraction (all kernels)", alg, ms)}
    if not args.no_cpu:
        from oracle import oracle as O
        import numpy as np
        h = O.Hypergraph(inst.n, inst.eptr, inst.pins, inst.c, inst.w)
        t0 = time.perf_counter()
        mp_o, hc = O.contract(h, cl)
        dt = time.perf_counter() - t0
        assert (nc, mc, pc) == (hc.n, hc.m, hc.P), "coarse sizes differ from the oracle"
        mp, cv, ce, cpn, cw = (x.cpu().numpy() for x in out.views())
        for got, want, what in ((mp, mp_o, "map"), (cv, hc.c, "vertex weights"),
                                (ce, hc.eptr, "net offsets"), (cpn, hc.pins, "pins"),
                                (cw, hc.w, "net weights")):
            assert np.array_equal(got, want), "contraction %s differ from the oracle" % what
        res["cpu_baseline"] = {"value": inst.P / dt, "unit": "pins/s", "cores": 1,
                               "kind": "oracle", "host": host_info(),
                               "sample": "the whole contraction, once (equal to the GPU's "
                                         "output)"}
    g.free()
    return res


def copy_bandwidth(torch, dev, nbytes=1 << 30, reps=5):
    """A plain device-to-device copy of `nbytes` on the same GPU, as a
    measured reference beside the 8 TB/s peak: (read + write) bytes / time."""
    src = torch.ones(nbytes // 4, dtype=torch.int32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    xs = []
    for _ in range(reps):
        a, b = _events(torch)
        a.record()
        dst.copy_(src)
        b.record()
        b.synchronize()
        xs.append(a.elapsed_time(b))
    del src, dst
    ms = percentile(xs, 50)
    return {"bytes": 2 * nbytes, "ms": ms, "gbs": 2 * nbytes / (ms / 1e3) / 1e9}


def oracle_rounds(inst, ks, plan):
    """The oracle on the host (one thread): for each k, plan[k] LP rounds
    from the workload's start.  Returns ({k: (part, records)}, baseline)."""
    import numpy as np
    import synth
    from oracle import oracle as O
    h = O.Hypergraph(inst.n, inst.eptr, inst.pins, inst.c, inst.w)
    h.incidence()
    out, t_total, pin_rounds = {}, 0.0, 0
    for k in ks:
        ik = synth.with_k(inst, k)
        L = O.lmax(O.total_vertex_weight(h), k, inst.eps)
        part = ik.part.copy()
        elig = np.ones(inst.n, np.uint8)
        recs = []
        for _ in range(plan[k]):
            t0 = time.perf_counter()
            part, elig, _, st = O.lp_round(h, k, L, part, elig)
            t_total += time.perf_counter() - t0
            pin_rounds += inst.P
            recs.append(st)
        out[k] = (part, recs)
    base = {"value": pin_rounds / t_total, "unit": "pins/s", "cores": 1, "kind": "oracle",
            "sample": "the first %s LP rounds at k = %s of the same instance (%d pins), "
                      "single-threaded C oracle, %.1f s; every round record and the partition "
                      "after the last sampled round equal the GPU's"
                      % ("/".join(str(plan[k]) for k in ks), "/".join(map(str, ks)), inst.P,
                         t_total),
            "seconds": t_total, "host": host_info()}
    return out, base


def plain_workload(args, H, dev, inst, ks, rounds, label, cpu_plan, roofline=True):
    """One plain workload: a step is load + for every k (pin counts, `rounds`
    LP rounds, all k-way gains, km1), timed over args.steps steps with the
    inputs resident in HBM.  Value = len(ks) x rounds x P pins per step over
    the step time.  Beside it: per-phase and whole-round rooflines from the
    round records over the library's per-phase HIP events, per-round
    latency, the recorded-graph refine time and the oracle on a sample of
    the same rounds, checked record by record."""
    import numpy as np
    import torch
    import synth
    n, m, P = inst.n, inst.m, inst.P
    parts = {k: torch.as_tensor(synth.with_k(inst, k).part).to(dev) for k in ks}
    eptr = torch.as_tensor(inst.eptr).to(dev)
    pins = torch.as_tensor(inst.pins).to(dev)
    c = torch.as_tensor(inst.c).to(dev)
    w = torch.as_tensor(inst.w).to(dev)
    kmax = max(ks)
    ws_bytes = H.hg_workspace_size(n, m, P, kmax)
    bufs = (torch.empty(n + 1, dtype=torch.int64, device=dev),
            torch.empty(P, dtype=torch.int32, device=dev),
            torch.empty(ws_bytes, dtype=torch.uint8, device=dev))
    g0 = H.hg_load_csr(n, eptr, pins, c, w, k_max=kmax, device=dev, out=bufs)
    states = {k: H.State(g0, k, parts[k]) for k in ks}
    g0.free()
    stats = {k: torch.zeros(rounds * H.STATS_WORDS, dtype=torch.int64, device=dev) for k in ks}
    gains = torch.empty(n * kmax, dtype=torch.int64, device=dev)
    km1_out = torch.empty(1, dtype=torch.int64, device=dev)
    phase_ms = {p: 0.0 for p in H.HG_PHASES}
    timed_rounds = [0]

    def step(marks):
        # the step's graph handle is returned, not freed: reading its phase
        # marks and freeing it wait for the GPU, which the timed loop leaves
        # to after its last step (the next load reuses the same buffers in
        # stream order).  Phase marks (HIP events around the select, the
        # approval and the finalize of every round) are recorded when asked:
        # on the last timed step, a sample of the same work, so that the
        # marks' own cost (a few microseconds of idle GPU each) stays out of
        # the other steps
        g = H.hg_load_csr(n, eptr, pins, c, w, k_max=kmax, device=dev, out=bufs)
        H.hg_timing_enable(g, marks)
        for k in ks:
            st = states[k]
            st.part.copy_(parts[k])
            H.hg_refine(g, st, inst.eps, rounds, stats[k], use_graph=False)
            H.hg_gains(g, k, st.part, st.netstate, gains=gains[:n * k])
            H.hg_km1(g, k, st.netstate, out=km1_out)
        return g

    def retire(g, collect):
        ms, r = H.hg_timing_collect(g)     # waits for the step's last round
        if collect:
            for p in ms:
                phase_ms[p] += ms[p]
            timed_rounds[0] += r
        g.free()

    print("%s: warmup ..." % label, file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        retire(step(True), False)
    torch.cuda.synchronize()
    print("%s: timing %d steps ..." % (label, args.steps), file=sys.stderr, flush=True)
    e0, e1 = _events(torch)
    t0 = time.perf_counter()
    e0.record()
    done = [step(i == args.steps - 1) for i in range(args.steps)]
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for g in done:
        retire(g, True)
    gpu_ms = e0.elapsed_time(e1)
    elapsed = max(wall, gpu_ms / 1e3)
    ms_per_step = elapsed * 1e3 / args.steps
    value = len(ks) * rounds * P * args.steps / elapsed
    per_k = {k: H.stats_to_dicts(stats[k]) for k in ks}
    final_parts = {k: states[k].part.cpu().numpy() for k in ks}
    for k in ks:
        for s in per_k[k]:
            assert s["km1_delta"] == s["km1_delta_recomputed"], "attributed km1 mismatch"

    # rooflines: bytes of the step's rounds (records) over the phase times
    launches = len(ks) * rounds
    assert timed_rounds[0] == launches, "phase timing lost rounds"
    phase_bytes = {p: sum(f(s, n, k) for k in ks for s in per_k[k]) / launches
                   for p, f in PHASE_BYTES.items()}
    phase_avg = {p: phase_ms[p] / timed_rounds[0] for p in H.HG_PHASES}
    phases = {p: roofline_of(p, phase_bytes[p], phase_avg[p]) for p in H.HG_PHASES}
    round_ms = sum(phase_avg.values())
    whole = roofline_of("LP round (select + approve/apply + finalize)",
                        sum(phase_bytes.values()), round_ms)

    # per-k phase times from an untimed profile pass (same kernels)
    g = H.hg_load_csr(n, eptr, pins, c, w, k_max=kmax, device=dev, out=bufs)
    per_k_out = {}
    for k in ks:
        st = states[k]
        H.hg_timing_enable(g, True)
        for _ in range(args.latency_reps):
            st.part.copy_(parts[k])
            H.hg_refine(g, st, inst.eps, rounds, stats[k], use_graph=False)
        ms, r = H.hg_timing_collect(g)
        H.hg_timing_enable(g, False)
        avg = {p: ms[p] / r for p in H.HG_PHASES}
        by = {p: sum(f(s, n, k) for s in per_k[k]) / rounds for p, f in PHASE_BYTES.items()}
        per_k_out["k%d" % k] = {
            "phase_ms_per_round": avg,
            "phase_frac": {p: roofline_of(p, by[p], avg[p])["frac"] for p in H.HG_PHASES},
            "round_frac": roofline_of("round", sum(by.values()), sum(avg.values()))["frac"],
            "round_bytes": sum(by.values()),
            "records": per_k[k],
        }

    # per-round latency: each round timed alone (events around hg_lp_round)
    lat = {}
    one = torch.zeros(H.STATS_WORDS, dtype=torch.int64, device=dev)
    for k in ks:
        st = states[k]
        L = H.hg_max_block_weight(g, k, inst.eps)
        xs, first = [], []
        for _ in range(args.latency_reps):
            st.part.copy_(parts[k])
            H.hg_compute_pincounts(g, st)
            st.eligible.fill_(1)
            for r in range(rounds):
                a, b = _events(torch)
                a.record()
                H.hg_lp_round(g, st, L, one, moved=False)
                b.record()
                b.synchronize()
                xs.append(a.elapsed_time(b))
                if r == 0:
                    first.append(xs[-1])
        lat["k%d" % k] = {"p50_ms": percentile(xs, 50), "p99_ms": percentile(xs, 99),
                          "round1_p50_ms": percentile(first, 50),
                          "pins_per_s_p50": P / (percentile(xs, 50) / 1e3)}
    # recorded hipGraph replay of the same refinement
    graph_ms = {}
    for k in ks:
        st = states[k]
        xs = []
        for _ in range(args.latency_reps + 1):
            st.part.copy_(parts[k])
            a, b = _events(torch)
            a.record()
            H.hg_refine(g, st, inst.eps, rounds, stats[k], use_graph=True)
            b.record()
            b.synchronize()
            xs.append(a.elapsed_time(b))
        graph_ms["k%d" % k] = percentile(xs[1:], 50)       # first call records the graph
        assert H.stats_to_dicts(stats[k]) == per_k[k], "graph replay differs"

    out = {
        "value": value,
        "unit": "pins/s",
        "ms_per_step": ms_per_step,
        "n": n, "m": m, "P": P, "k": list(ks), "rounds": rounds, "eps": inst.eps,
        "roofline": {
            "kernel": "k_select_light (LP select sweep)",
            "bound": "hbm",
            "achieved": phases["select"]["achieved"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": phases["select"]["frac"],
            "avg_launch_us": phase_avg["select"] * 1e3,
            "alg_bytes_per_launch": phase_bytes["select"],
            "round": whole,
            "phases": phases,
        },
        "per_k": per_k_out,
        "round_latency": lat,
        "graph_refine_ms": graph_ms,
        "km1_final": {"k%d" % k: per_k[k][-1]["km1_after"] for k in ks},
    }
    if not roofline:
        out["roofline"]["note"] = ("launch-bound instance (about a megabyte per round): "
                                   "no roofline claim")

    if not args.no_cpu:
        print("%s: oracle rounds ..." % label, file=sys.stderr, flush=True)
        want, base = oracle_rounds(inst, ks, cpu_plan)
        for k in ks:
            part_o, recs_o = want[k]
            R = len(recs_o)
            for r in range(R):
                got = dict(per_k[k][r])
                got.pop("km1_delta_recomputed")
                assert got == recs_o[r], "%s k=%d round %d differs from the oracle" % (
                    label, k, r)
            if R == rounds:
                got_part = final_parts[k]
            else:
                st = states[k]
                st.part.copy_(parts[k])
                H.hg_refine(g, st, inst.eps, R, stats[k][:R * H.STATS_WORDS], use_graph=False)
                got_part = st.part.cpu().numpy()
            assert np.array_equal(got_part, part_o), "%s k=%d partition differs" % (label, k)
        out["cpu_baseline"] = base
        out["check"] = ("round records of the timed steps equal the oracle's for the sampled "
                        "rounds, and the partitions after them")
    g.free()
    del states, bufs, gains
    torch.cuda.empty_cache()
    return out


def headline(args, rec, workload, config_extra):
    """The benchmark line's top-level fields from one plain workload."""
    out = {
        "metric": METRIC,
        "value": rec["value"],
        "unit": "pins/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": rec["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": dict({"workload": workload, "parallelism": "single GPU"}, **config_extra),
        "roofline": rec["roofline"],
    }
    if "cpu_baseline" in rec:
        out["cpu_baseline"] = rec["cpu_baseline"]
    return out


def attach_traffic(roof, profile):
    """Measured HBM-side bytes (committed counter summary) beside the
    algorithmic ones: the select per launch, the approve and finalize phases
    per round, and the whole round."""
    roof["traffic"] = measured_traffic(profile, "select")
    roof["traffic_unit"] = ("bytes per launch: L2-to-fabric read and write requests by size "
                            "(32/64/128 B) from rocprofv3 counters, profiles/" + profile)
    tot = roof["traffic"]
    for p in ("approve", "finalize"):
        t = measured_traffic(profile, p)
        roof["phases"][p]["traffic"] = t
        tot = None if tot is None or t is None else tot + t
    roof["phases"]["select"]["traffic"] = roof["traffic"]
    roof["round"]["traffic"] = tot


def plain_legs(args, H, dev):
    """The plain workloads: the VLSI-like netlist (the headline), the
    sparse matrix and the tiny instance."""
    import synth
    which = set(args.plain_workloads.split(","))
    out = {"metric": METRIC}
    if "vlsi" in which:
        out = vlsi_headline(args, H, dev)
    if "sparse" in which:
        sp = sparse_instance()
        srec = plain_workload(args, H, dev, sp, KS, ROUNDS, "sparse",
                              {8: ROUNDS, 64: args.cpu_rounds_k64})
        attach_traffic(srec["roofline"], "plain_sparse_matrix_traffic.md")
        srec["config"] = ("sparse-matrix row-net hypergraph 1M x 1M (%d pins), k = 8 and k = 64, "
                          "eps = 0.03, 10 synchronous LP rounds per k; one step = load + (pin "
                          "counts + 10 rounds + gains + km1) per k" % sp.P)
        out["sparse_matrix"] = srec
        del sp
    if "tiny" in which:
        tiny = synth.tiny_plain()
        trec = plain_workload(args, H, dev, tiny, (2,), 5, "tiny", {2: 5}, roofline=False)
        trec["config"] = "tiny power-law hypergraph n = m = 10,000 (%d pins), k = 2, 5 rounds" % tiny.P
        out["tiny"] = trec
    return out


def vlsi_headline(args, H, dev):
    """The headline line: the VLSI-like netlist at its own k."""
    import torch
    import synth
    print("generating the VLSI-like netlist ...", file=sys.stderr, flush=True)
    vl = synth.vlsi_grid()
    rec = plain_workload(args, H, dev, vl, (vl.k,), ROUNDS, "vlsi", {vl.k: args.cpu_rounds})
    attach_traffic(rec["roofline"], "plain_vlsi_traffic.md")
    rec["roofline"]["copy_reference"] = copy_bandwidth(torch, dev)
    out = headline(args, rec, "VLSI-like netlist: 2000 x 2000 grid, n = %d cells, m = %d nets, "
                   "%d pins, k = %d, eps = 0.03, 10 synchronous LP rounds; one step = load + "
                   "pin counts + 10 rounds + gains + km1" % (vl.n, vl.m, vl.P, vl.k),
                   {"n": vl.n, "m": vl.m, "P": vl.P, "k": [vl.k], "rounds": ROUNDS,
                    "eps": vl.eps, "seed": 3})
    out["vlsi"] = {x: rec[x] for x in ("per_k", "round_latency", "graph_refine_ms",
                                        "km1_final", "check") if x in rec}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-rounds", type=int, default=4,
                    help="oracle rounds sampled on the VLSI-like netlist")
    ap.add_argument("--cpu-rounds-k64", type=int, default=3,
                    help="oracle rounds sampled on the sparse matrix at k = 64 (all 10 at k = 8)")
    ap.add_argument("--latency-reps", type=int, default=5)
    ap.add_argument("--legs", default="plain,batched,served,monotone,cached,rebalance,contract",
                    help="comma list of plain, batched, served, monotone, cached, rebalance, "
                         "contract")
    ap.add_argument("--plain-workloads", default="vlsi,sparse,tiny",
                    help="comma list of the plain leg's workloads: vlsi (the headline line), "
                         "sparse, tiny")
    ap.add_argument("--mono-reps", type=int, default=3)
    ap.add_argument("--served-seconds", type=float, default=60.0,
                    help="length of the open-loop request trace (60 s: about 12,000 requests)")
    ap.add_argument("--batch-count", type=int, default=BATCH_COUNT)
    ap.add_argument("--batch-reps", type=int, default=5)
    ap.add_argument("--batch-cpu-s", type=float, default=8.0)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="also run one plain device-to-device copy of MIB MiB (a known "
                         "byte count for scaling HBM traffic counters)")
    args = ap.parse_args()
    if args.steps < 1 or args.warmup < 0:
        print("bench.py needs --steps >= 1 and --warmup >= 0", file=sys.stderr)
        sys.exit(2)
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
    out = plain_legs(args, H, dev) if "plain" in legs else {"metric": METRIC}
    if args.calibrate_copy > 0:
        nb = args.calibrate_copy << 20
        src = torch.ones(nb // 4, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["calibrate_copy_bytes"] = nb
        del src, dst
    if "batched" in legs:
        torch.cuda.empty_cache()
        out["batched"] = batched_leg(args, H, dev)
    if "served" in legs:
        torch.cuda.empty_cache()
        out["served"] = served_leg(args, H, dev)
    if "monotone" in legs:
        torch.cuda.empty_cache()
        print("monotone rounds ...", file=sys.stderr, flush=True)
        out["monotone"] = monotone_leg(args, H, dev)
    if "cached" in legs:
        torch.cuda.empty_cache()
        print("gain-cache rounds ...", file=sys.stderr, flush=True)
        out["cached"] = cached_leg(args, H, dev)
    if "rebalance" in legs:
        torch.cuda.empty_cache()
        print("rebalancing rounds ...", file=sys.stderr, flush=True)
        out["rebalance"] = rebalance_leg(args, H, dev)
    if "contract" in legs:
        torch.cuda.empty_cache()
        print("contraction ...", file=sys.stderr, flush=True)
        out["contract"] = contract_leg(args, H, dev)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
