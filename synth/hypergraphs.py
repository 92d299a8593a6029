"""Seeded synthetic hypergraphs shaped like the paper's benchmark instances.

The paper evaluates on SuiteSparse row-net matrices, ISPD98/DAC2012 VLSI
netlists and SAT14 formulas (section "Experiments", subsection "Instances").
None of those files are available here, so these generators stand in for them
with the same shapes: power-law net sizes, banded sparse-matrix rows, and
grid-local VLSI nets with a few global nets.

This module holds input generation only: random draws, shapes and start
partitions.  It contains none of the refinement arithmetic and is shared by the
oracle side and the HIP side of the tests and the benchmark.

All draws use numpy's PCG64 (``np.random.default_rng(seed)``) in the order the
docstrings state, so an instance is a pure function of its seed and sizes.
Pins inside a net are stored in increasing vertex order.
"""
import numpy as np

from dataclasses import dataclass, field


@dataclass
class Instance:
    """A hypergraph in net-CSR form plus a start partition and run settings."""
    name: str
    n: int
    eptr: np.ndarray            # int64[m+1]
    pins: np.ndarray            # int32[P]
    c: np.ndarray               # int32[n] vertex weights
    w: np.ndarray               # int32[m] net weights
    part: np.ndarray            # int32[n] start partition
    k: int
    eps: float = 0.03
    rounds: int = 5
    meta: dict = field(default_factory=dict)

    @property
    def m(self):
        return int(self.eptr.shape[0] - 1)

    @property
    def P(self):
        return int(self.eptr[-1])


def _csr_from_sizes(sizes):
    eptr = np.zeros(sizes.shape[0] + 1, np.int64)
    np.cumsum(sizes, out=eptr[1:])
    return eptr


def _slots_of(eptr, nets):
    """Pin positions of the given nets, net after net."""
    sz = eptr[nets + 1] - eptr[nets]
    before = np.concatenate(([0], np.cumsum(sz)[:-1]))
    return np.repeat(eptr[nets] - before, sz) + np.arange(int(sz.sum()), dtype=np.int64)


def _distinct_within_nets(rng, eptr, draw):
    """Draw pins net by net so that no vertex repeats inside a net.

    ``draw(rng, slot_net_ids)`` returns one candidate vertex per pin slot.  All
    slots are drawn once; slots whose value repeats an earlier slot of the same
    net are redrawn (in increasing slot order), until no net holds a repeated
    vertex.  Each net is finally sorted.
    """
    m = eptr.shape[0] - 1
    sizes = np.diff(eptr)
    net_of = np.repeat(np.arange(m, dtype=np.int64), sizes)
    vals = draw(rng, net_of).astype(np.int64)
    todo = np.arange(m, dtype=np.int64)           # nets still to check
    while todo.size:
        # slots of the nets to check
        slot = _slots_of(eptr, todo)
        owner = net_of[slot]
        key = owner * (1 << 32) + vals[slot]
        order = np.argsort(key, kind="stable")
        ks = key[order]
        dup = np.zeros(ks.shape[0], bool)
        dup[1:] = ks[1:] == ks[:-1]
        if not dup.any():
            break
        redo = np.sort(slot[order[dup]])
        vals[redo] = draw(rng, net_of[redo])
        todo = np.unique(net_of[redo])
    # sort pins inside every net
    key = net_of * (1 << 32) + vals
    vals = vals[np.argsort(key, kind="stable")]
    return vals.astype(np.int32)


def _power_law_sizes(rng, count, lo, hi, exponent=2.5):
    s = np.arange(lo, hi + 1, dtype=np.int64)
    p = s.astype(np.float64) ** (-exponent)
    p /= p.sum()
    return rng.choice(s, size=count, p=p)


def random_power_law(seed, n, m, k, lo=2, hi=64, unit=True, rounds=5, eps=0.03,
                     name=None):
    """Random hypergraph with power-law net sizes (the tiny plain workload).

    Draw order: net sizes ~ P(s) proportional to s^-2.5 on [lo, min(hi, n)];
    pins uniform over [0, n), distinct per net; start partition
    Pi(v) = perm[v] mod k for a uniform random permutation perm.  With
    ``unit=False`` vertex weights ~ U{1..8} and net weights ~ U{1..4} are drawn
    last.
    """
    rng = np.random.default_rng(seed)
    hi = min(hi, n)
    lo = min(lo, hi)
    sizes = _power_law_sizes(rng, m, lo, hi)
    eptr = _csr_from_sizes(sizes)
    pins = _distinct_within_nets(rng, eptr, lambda r, nets: r.integers(0, n, nets.shape[0]))
    perm = rng.permutation(n)
    part = (perm % k).astype(np.int32)
    meta = {"seed": seed, "perm": perm}
    if unit:
        c = np.ones(n, np.int32)
        w = np.ones(m, np.int32)
    else:
        c = rng.integers(1, 9, n).astype(np.int32)
        w = rng.integers(1, 5, m).astype(np.int32)
    return Instance(name or "powerlaw-n%d-m%d-k%d" % (n, m, k), n, eptr, pins, c, w, part,
                    k, eps, rounds, meta)


def tiny_plain(seed=1):
    """Tiny plain workload: n = m = 10,000, power-law sizes in [2,64], k = 2,
    unit weights, random balanced start, eps = 0.03, 5 rounds (seed 1)."""
    return random_power_law(seed, 10_000, 10_000, 2, rounds=5, name="tiny-10k-k2")


def sparse_matrix(k, seed=2, rows=1_000_000, cols=1_000_000, band=5_000, rounds=10):
    """Row-net hypergraph of a random sparse matrix (rows are nets, columns are
    vertices), about 10 pins per row.

    Draw order: row lengths round(LogNormal(mu, 1.0)) with mu = ln 10 - 1/2 (so
    the mean is 10), clamped to [1, 2000]; then per pin slot a uniform U(0,1)
    chooses band (< 0.7) or global, and a column is drawn uniform in
    [row - band, row + band] clipped to the matrix, or uniform over all
    columns; repeated columns in a row are redrawn the same way; then the start
    permutation.  Vertex weight = max(1, column degree), net weight 1,
    Pi(v) = perm[v] mod k.
    """
    rng = np.random.default_rng(seed)
    sigma = 1.0
    mu = np.log(10.0) - sigma * sigma / 2
    lens = np.rint(rng.lognormal(mu, sigma, rows)).astype(np.int64)
    lens = np.clip(lens, 1, 2000)
    eptr = _csr_from_sizes(lens)

    def draw(r, nets):
        cnt = nets.shape[0]
        local = r.random(cnt) < 0.7
        lo = np.maximum(nets - band, 0)
        hi = np.minimum(nets + band, cols - 1)
        u = r.random(cnt)
        band_col = lo + np.floor(u * (hi - lo + 1)).astype(np.int64)
        glob_col = r.integers(0, cols, cnt)
        return np.where(local, band_col, glob_col)

    pins = _distinct_within_nets(rng, eptr, draw)
    perm = rng.permutation(cols)
    deg = np.bincount(pins, minlength=cols)
    c = np.maximum(deg, 1).astype(np.int32)
    w = np.ones(rows, np.int32)
    part = (perm % k).astype(np.int32)
    return Instance("sparse-matrix-1Mx1M-k%d" % k, cols, eptr, pins, c, w, part, k, 0.03,
                    rounds, {"seed": seed, "perm": perm})


def with_k(inst, k):
    """The same hypergraph with its start partition for k blocks: perm[v] mod
    k for the instances whose start is a random permutation, horizontal
    strips floor(y * k / height) for the grid netlists."""
    if "perm" in inst.meta:
        part = (inst.meta["perm"] % k).astype(np.int32)
    else:
        side, height = inst.meta["side"], inst.meta["height"]
        y = np.arange(inst.n, dtype=np.int64) // side
        part = (y * k // height).astype(np.int32)
    name = inst.name.rsplit("-k", 1)[0] + "-k%d" % k
    return Instance(name, inst.n, inst.eptr, inst.pins, inst.c, inst.w, part, k, inst.eps,
                    inst.rounds, dict(inst.meta))


def vlsi_grid(seed=3, side=2000, height=2000, m=4_200_000, k=16, rounds=10):
    """VLSI-like netlist on a side x height grid of cells (v = y*side + x).

    Draw order: per net a U(0,1) picks the size class (< 0.9: uniform{2..5},
    else uniform{6..200}) and the size; a second U(0,1) marks 1% of nets
    global; local nets draw a 16x16 window origin uniform in
    [0, side-16] x [0, height-16] and take distinct cells of that window
    (redrawing repeats for nets of at most 16 pins, a random-key shuffle of
    the 256 window cells for larger ones); global nets take distinct cells
    uniform over the grid; vertex weights ~ U{1..8}; net weights 1.  Start
    partition: horizontal strips, Pi(v) = floor(y * k / height).
    """
    rng = np.random.default_rng(seed)
    n = side * height
    big = rng.random(m) >= 0.9
    small_sz = rng.integers(2, 6, m)
    big_sz = rng.integers(6, 201, m)
    sizes = np.where(big, big_sz, small_sz).astype(np.int64)
    glob = rng.random(m) < 0.01
    ox = rng.integers(0, side - 16 + 1, m)
    oy = rng.integers(0, height - 16 + 1, m)
    eptr = _csr_from_sizes(sizes)

    # nets drawn by redraw-on-repeat: global nets and local nets of <= 16 pins
    pins = np.empty(int(eptr[-1]), np.int32)
    by_redraw = glob | (sizes <= 16)

    def draw(r, nets):
        cnt = nets.shape[0]
        cell = r.integers(0, 256, cnt)
        anywhere = r.integers(0, n, cnt)
        local_v = (oy[nets] + cell // 16) * side + (ox[nets] + cell % 16)
        return np.where(glob[nets], anywhere, local_v)

    sel = np.nonzero(by_redraw)[0]
    sub_eptr = _csr_from_sizes(sizes[sel])
    sub_pins = _distinct_within_nets(rng, sub_eptr, lambda r, nets: draw(r, sel[nets]))
    pins[_slots_of(eptr, sel)] = sub_pins

    # large local nets: first |e| cells of a random order of the 256 window cells
    rest = np.nonzero(~by_redraw)[0]
    chunk = 32768
    for s0 in range(0, rest.shape[0], chunk):
        nets = rest[s0:s0 + chunk]
        keys = rng.random((nets.shape[0], 256))
        order = np.argsort(keys, axis=1, kind="stable")
        s = sizes[nets]
        take = np.arange(256)[None, :] < s[:, None]
        cells = np.sort(np.where(take, order, 256), axis=1)
        cells = cells[np.arange(256)[None, :] < s[:, None]]      # row-major = net order
        owner = np.repeat(nets, s)
        pins[_slots_of(eptr, nets)] = (oy[owner] + cells // 16) * side + (ox[owner] + cells % 16)
    c = rng.integers(1, 9, n).astype(np.int32)
    w = np.ones(m, np.int32)
    y = np.arange(n, dtype=np.int64) // side
    part = (y * k // height).astype(np.int32)
    return Instance("vlsi-%dx%d-m%d-k%d" % (side, height, m, k), n, eptr, pins, c, w, part,
                    k, 0.03, rounds, {"seed": seed, "side": side, "height": height})


def _batch_member(args):
    seed, n, m, k, rounds, i = args
    return random_power_law(seed, n, m, k, hi=64, unit=True, rounds=rounds,
                            name="batch%d-n%d-k%d" % (i, n, k))


def batch_instances(seed=4, count=512, n_lo=1_000, n_hi=500_000, ks=(2, 4, 8, 32, 128),
                    rounds=8, workers=1):
    """Many independent power-law hypergraphs of uneven sizes (the batched
    workload: 512 instances, 8 rounds each).

    Draw order (one generator seeded with `seed`): for all instances, n =
    round(exp(U(ln n_lo, ln n_hi))); then m = round(n * U(0.8, 1.2)); then k
    uniform over `ks`; then a 63-bit seed per instance.  Instance i is
    random_power_law(seed_i, n_i, m_i, k_i) with net sizes in [2, min(64, n)],
    unit weights and Pi(v) = perm[v] mod k.  `workers` > 1 builds the
    instances in that many processes (same result: each depends on its own
    seed only).
    """
    rng = np.random.default_rng(seed)
    ns = np.rint(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi), count))).astype(np.int64)
    ms = np.maximum(np.rint(ns * rng.uniform(0.8, 1.2, count)), 1).astype(np.int64)
    kk = np.asarray(ks, np.int64)[rng.integers(0, len(ks), count)]
    seeds = rng.integers(0, 2 ** 63 - 1, count, dtype=np.int64)
    args = [(int(seeds[i]), int(ns[i]), int(ms[i]), int(kk[i]), rounds, i) for i in range(count)]
    if workers > 1:
        from concurrent.futures import ProcessPoolExecutor
        import multiprocessing as mp
        with ProcessPoolExecutor(workers, mp_context=mp.get_context("fork")) as ex:
            return list(ex.map(_batch_member, args, chunksize=4))
    return [_batch_member(a) for a in args]


@dataclass
class Request:
    """One job of a served trace: its scheduled arrival, the pool instance it
    refines and its k (the start partition is the instance's for that k)."""
    arrival_s: float
    big: bool
    pool: int
    k: int
    rounds: int
    eps: float = 0.03


def served_trace(seed=5, rate=200.0, seconds=60.0, big_prob=0.05, ks=(2, 4, 8, 32, 128),
                 rounds=10, small_pool=256, big_pool=2):
    """Open-loop request trace: Poisson arrivals at `rate` per second for
    `seconds`; each request is w.p. `big_prob` a grid netlist with n = 2M
    (2000 x 1000 cells, m = 2.1M) and otherwise a hypergraph of the batched
    workload's size distribution; k uniform over `ks`; `rounds` rounds.

    Draw order (one generator seeded with `seed`): inter-arrival gaps
    Exp(1/rate) until the horizon; then per request a U(0,1) for big-vs-small,
    a pool index and an index into `ks`.  Requests refine instances from a
    pool (`small_pool` of the batched distribution, seed + 1; `big_pool`
    netlists, seeds seed + 2, ...), so a trace of thousands of requests needs
    only a few hundred distinct hypergraphs; see served_pool.
    """
    rng = np.random.default_rng(seed)
    gaps = []
    t = 0.0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= seconds:
            break
        gaps.append(t)
    cnt = len(gaps)
    big = rng.random(cnt) < big_prob
    small_idx = rng.integers(0, small_pool, cnt)
    big_idx = rng.integers(0, big_pool, cnt)
    kidx = rng.integers(0, len(ks), cnt)
    return [Request(gaps[i], bool(big[i]), int(big_idx[i] if big[i] else small_idx[i]),
                    int(ks[kidx[i]]), rounds) for i in range(cnt)]


def served_pool(seed=5, small_pool=256, big_pool=2, workers=1):
    """The instances a served trace draws from: (small, big) lists."""
    small = batch_instances(seed=seed + 1, count=small_pool, rounds=10, workers=workers)
    seeds = [seed + 2 + i for i in range(big_pool)]
    if workers > 1 and big_pool > 1:
        from concurrent.futures import ProcessPoolExecutor
        import multiprocessing as mp
        with ProcessPoolExecutor(min(workers, big_pool), mp_context=mp.get_context("fork")) as ex:
            big = list(ex.map(_big_netlist, seeds))
    else:
        big = [_big_netlist(s) for s in seeds]
    return small, big


def _big_netlist(seed):
    return vlsi_grid(seed=seed, side=2000, height=1000, m=2_100_000, k=16, rounds=10)


def neighbour_clusters(inst, seed=6, join=0.5):
    """A seeded clustering of the shape one coarsening pass produces: a
    random `join` share of the vertices names a neighbour (another pin of one
    of its nets, drawn at random) as its cluster id; the others keep their
    own id.  Ids are vertex ids, so most of [0, n) is unused."""
    rng = np.random.default_rng(seed)
    n, eptr, pins = inst.n, inst.eptr, inst.pins
    sizes = np.diff(eptr)
    net_of = np.repeat(np.arange(inst.m), sizes)
    # every vertex picks the incident net of its highest-priority pin slot
    prio = rng.random(pins.shape[0])
    order = np.argsort(pins + prio)          # by vertex, then by priority
    last = np.ones(pins.shape[0], bool)
    last[:-1] = pins[order][1:] != pins[order][:-1]
    pick = np.full(n, -1, np.int64)
    pick[pins[order][last]] = net_of[order][last]
    cluster = np.arange(n, dtype=np.int32)
    has = pick >= 0
    e = pick[has]
    first = pins[eptr[e]]
    second = pins[np.minimum(eptr[e] + 1, eptr[e + 1] - 1)]
    verts = np.nonzero(has)[0]
    partner = np.where(first != verts, first, second)
    joins = rng.random(verts.shape[0]) < join
    cluster[verts[joins]] = partner[joins]
    return cluster


def describe(inst):
    sizes = np.diff(inst.eptr)
    deg = np.bincount(inst.pins, minlength=inst.n)
    return {
        "name": inst.name, "n": inst.n, "m": inst.m, "P": inst.P, "k": inst.k,
        "mean_net_size": float(sizes.mean()), "max_net_size": int(sizes.max()),
        "single_pin_nets": int((sizes == 1).sum()),
        "mean_degree": float(deg.mean()), "max_degree": int(deg.max()),
        "total_vertex_weight": int(inst.c.astype(np.int64).sum()),
    }
