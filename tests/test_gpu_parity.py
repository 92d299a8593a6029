"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Everything is integer, so every comparison is exact (bit-identical arrays and
statistics).  Inputs are seeded synthetic hypergraphs sized so that the oracle
finishes in seconds while spanning several 4096-vertex approval tiles with a
ragged tail, every bitset width (k up to 256), weighted and unit inputs, and
the wavefront path for heavy vertices (w(I(v)) > 255).
"""
import numpy as np
import pytest

import synth
from oracle import oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2010_10272_amd import hgref
    return hgref


def _oracle_hg(inst):
    return O.Hypergraph(inst.n, inst.eptr, inst.pins, inst.c, inst.w)


def _bits_to_sets(words, k):
    """uint32 words [m, W] -> boolean [m, k]."""
    w = np.asarray(words, dtype=np.uint32)
    out = np.zeros((w.shape[0], k), bool)
    for i in range(k):
        out[:, i] = (w[:, i // 32] >> np.uint32(i % 32)) & 1
    return out


def _check_state(H, g, st, h, k, part_np):
    """Device state (phi, netstate, block_w) equals the oracle's recomputation
    from part_np."""
    phi_o = O.pin_counts(h, part_np, k)
    lam_o, _ = O.connectivity(phi_o, k)
    phi_g = st.phi.view(g.m, k).cpu().numpy()
    assert np.array_equal(phi_g, phi_o)
    w_g, lam_g, conn_g, single_g = (x.cpu().numpy() for x in H.decode_netstate(st.netstate, g.m, k))
    assert np.array_equal(lam_g, lam_o)
    assert np.array_equal(w_g, h.w if h.w is not None else np.ones(g.m, np.int32))
    assert np.array_equal(_bits_to_sets(conn_g, k), phi_o > 0)
    assert np.array_equal(_bits_to_sets(single_g, k), phi_o == 1)
    unit = h.w is None or bool((h.w == 1).all())
    if unit and k <= 64:
        # compact Lambda/S copy behind the records (maintained for unit nets)
        rw = H.hg_net_words(k)
        tail = st.netstate[g.m * rw:].cpu().numpy().astype(np.uint32)
        if k <= 16:
            lam_w = (tail & 0xffff)[:, None]
            s_w = (tail >> 16)[:, None]
        else:
            v = tail.reshape(g.m, -1)
            half = v.shape[1] // 2
            lam_w, s_w = v[:, :half], v[:, half:]
        assert np.array_equal(_bits_to_sets(lam_w, k), phi_o > 0)
        assert np.array_equal(_bits_to_sets(s_w, k), phi_o == 1)
    assert np.array_equal(st.block_w.cpu().numpy(), O.block_weights(h, part_np, k))
    return lam_o


def _hub_instance(seed, n, m, k, hub_deg, weighted):
    """Power-law hypergraph plus a few hub vertices in many nets, so that
    some vertices take the heavy (w(I(v)) > 255) path and some rows are long."""
    rng = np.random.default_rng(seed)
    base = synth.random_power_law(seed, n, m, k, hi=16, unit=not weighted)
    nets = [list(base.pins[base.eptr[e]:base.eptr[e + 1]]) for e in range(base.m)]
    hubs = [0, 1, n // 2]
    for hub in hubs:
        chosen = rng.choice(base.m, size=min(hub_deg, base.m), replace=False)
        for e in chosen:
            if hub not in nets[e]:
                nets[e].append(hub)
    for e in range(base.m):
        nets[e].sort()
    eptr = np.zeros(base.m + 1, np.int64)
    eptr[1:] = np.cumsum([len(x) for x in nets])
    pins = np.array([v for x in nets for v in x], np.int32)
    w = base.w
    if weighted:
        w = rng.integers(1, 300, base.m).astype(np.int32)
    return synth.Instance("hub-%d" % seed, n, eptr, pins, base.c, w, base.part, k, 0.03, 4)


def _cases():
    yield "tiny-10k-k2", lambda: synth.tiny_plain()
    for k, weighted in [(3, False), (5, True), (8, False), (16, True), (31, False), (33, True),
                        (64, False), (100, True), (128, False), (200, True), (256, False)]:
        yield ("plaw-k%d-%s" % (k, "w" if weighted else "u"),
               lambda k=k, weighted=weighted: synth.random_power_law(
                   1000 + k, 9000 + 37 * k, 8500 + 11 * k, k, hi=24, unit=not weighted,
                   rounds=4))
    # banded row-net matrices (net ids follow vertex ids)
    for k in (8, 32):
        yield ("band-k%d" % k, lambda k=k: synth.sparse_matrix(
            k, seed=40 + k, rows=40000, cols=40000, band=1500, rounds=4))
    # average degree 12 and more (the select sweep's eight-wide gathers)
    yield "vlsi-200x200-k16", lambda: synth.vlsi_grid(seed=11, side=200, height=200, m=42000,
                                                      k=16, rounds=4)
    yield "dense-k33-w", lambda: synth.random_power_law(77, 4000, 20000, 33, hi=40, unit=False,
                                                        rounds=4)
    yield "dense-k64-u", lambda: synth.random_power_law(78, 4000, 20000, 64, hi=40, unit=True,
                                                        rounds=4)
    yield "hub-k4-u", lambda: _hub_instance(7, 6000, 5000, 4, 300, False)
    yield "hub-k16-w", lambda: _hub_instance(8, 6000, 5000, 16, 400, True)
    yield "hub-k70-w", lambda: _hub_instance(9, 5000, 4000, 70, 500, True)


CASES = list(_cases())


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_load_pincounts_km1_gains(H, name, make):
    import torch
    inst = make()
    h = _oracle_hg(inst)
    k = inst.k
    g = H.hg_load_csr(inst.n, inst.eptr, inst.pins, inst.c, inst.w, k_max=k)
    vptr_o, vnets_o = O.incidence(h)
    assert np.array_equal(g.vptr.cpu().numpy(), vptr_o)
    assert np.array_equal(g.vnets[:inst.P].cpu().numpy(), vnets_o)
    info = H.hg_get_info(g)
    assert info["total_vertex_weight"] == int(inst.c.astype(np.int64).sum())
    assert info["total_net_weight"] == int(inst.w.astype(np.int64).sum())
    deg = np.diff(vptr_o)
    assert info["max_degree"] == int(deg.max())
    sizes = np.diff(inst.eptr)
    assert info["max_net_size"] == int(sizes.max())
    w = np.ones(inst.m, np.int64) if inst.w is None else inst.w.astype(np.int64)
    inc_w = np.array([w[vnets_o[vptr_o[v]:vptr_o[v + 1]]].sum() for v in range(inst.n)])
    assert info["max_incident_weight"] == int(inc_w.max())
    assert info["heavy_vertices"] == int((inc_w > 255).sum())
    st = H.State(g, k, inst.part)
    H.hg_compute_pincounts(g, st)
    torch.cuda.synchronize()
    lam_o = _check_state(H, g, st, h, k, inst.part)
    km1_o = O.km1(h, lam_o)
    assert int(st.km1.item()) == km1_o
    assert int(H.hg_km1(g, k, st.netstate).item()) == km1_o
    benefit = torch.empty(inst.n, dtype=torch.int64, device="cuda")
    gains, _ = H.hg_gains(g, k, st.part, st.netstate, benefit=benefit)
    gains_o, ben_o = O.gains(h, inst.part, k)
    assert np.array_equal(gains.view(inst.n, k).cpu().numpy(), gains_o)
    assert np.array_equal(benefit.cpu().numpy(), ben_o)
    H.hg_sync_status(g)


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_lp_rounds_bit_exact(H, name, make):
    import torch
    inst = make()
    h = _oracle_hg(inst)
    k = inst.k
    g = H.hg_load_csr(inst.n, inst.eptr, inst.pins, inst.c, inst.w, k_max=k)
    L = H.hg_max_block_weight(g, k, inst.eps)
    assert L == O.lmax(O.total_vertex_weight(h), k, inst.eps)
    st = H.State(g, k, inst.part)
    H.hg_compute_pincounts(g, st)
    part_o = inst.part.copy()
    elig_o = np.ones(inst.n, np.uint8)
    stats = torch.zeros(H.STATS_WORDS, dtype=torch.int64, device="cuda")
    for r in range(inst.rounds):
        H.hg_lp_round(g, st, L, stats)
        torch.cuda.synchronize()
        part_o, elig_o, moved_o, st_o = O.lp_round(h, k, L, part_o, elig_o)
        sg = H.stats_to_dicts(stats)[0]
        assert sg["km1_delta_recomputed"] == sg["km1_delta"], (r, sg)
        sg.pop("km1_delta_recomputed")
        assert sg == st_o, (r, sg, st_o)
        assert np.array_equal(st.part.cpu().numpy(), part_o), r
        assert np.array_equal(st.moved.cpu().numpy(), moved_o), r
        assert np.array_equal(st.eligible.cpu().numpy(), elig_o), r
        _check_state(H, g, st, h, k, part_o)
        assert int(st.km1.item()) == st_o["km1_after"]
    H.hg_sync_status(g)


@pytest.mark.parametrize("shift", [1, 2, 3])
def test_load_into_unaligned_incidence_buffer(H, shift):
    """A caller's incidence array that is 4-byte but not 16-byte aligned: the
    row starts then read it word by word; same rows as the oracle's."""
    import torch
    inst = synth.sparse_matrix(8, seed=70 + shift, rows=20000, cols=20000, band=800, rounds=2)
    h = _oracle_hg(inst)
    vptr = torch.empty(inst.n + 1, dtype=torch.int64, device="cuda")
    vnets_big = torch.empty(inst.P + 4, dtype=torch.int32, device="cuda")
    vnets = vnets_big[shift:shift + inst.P]
    assert vnets.data_ptr() % 16 != 0
    ws = torch.empty(H.hg_workspace_size(inst.n, inst.m, inst.P, 8), dtype=torch.uint8,
                     device="cuda")
    g = H.hg_load_csr(inst.n, inst.eptr, inst.pins, inst.c, inst.w, k_max=8,
                      out=(vptr, vnets, ws))
    vptr_o, vnets_o = O.incidence(h)
    assert np.array_equal(vptr.cpu().numpy(), vptr_o)
    assert np.array_equal(vnets.cpu().numpy(), vnets_o)
    H.hg_sync_status(g)


@pytest.mark.parametrize("use_graph", [False, True])
def test_refine_matches_oracle_and_replays(H, use_graph):
    import torch
    inst = synth.random_power_law(42, 20000, 19000, 16, hi=32, unit=False, rounds=6)
    h = _oracle_hg(inst)
    k = inst.k
    g = H.hg_load_csr(inst.n, inst.eptr, inst.pins, inst.c, inst.w, k_max=k)
    L = H.hg_max_block_weight(g, k, inst.eps)
    part_o, stats_o, km_o = O.refine(h, k, L, inst.rounds, inst.part)
    st = H.State(g, k, inst.part)
    stats = torch.zeros(inst.rounds * H.STATS_WORDS, dtype=torch.int64, device="cuda")
    for rep in range(3):            # replays of the recorded graph must all agree
        st.part.copy_(torch.as_tensor(inst.part))
        stats.zero_()
        H.hg_refine(g, st, inst.eps, inst.rounds, stats, use_graph=use_graph)
        torch.cuda.synchronize()
        assert np.array_equal(st.part.cpu().numpy(), part_o), rep
        got = H.stats_to_dicts(stats)
        for r in range(inst.rounds):
            assert got[r]["km1_delta_recomputed"] == got[r]["km1_delta"]
            got[r].pop("km1_delta_recomputed")
            assert got[r] == stats_o[r], (rep, r)
        assert int(st.km1.item()) == km_o
    H.hg_sync_status(g)


def test_tiny_plain_refine_5_rounds(H):
    """The tiny plain workload end to end (n = m = 10,000, k = 2, 5 rounds)."""
    import torch
    inst = synth.tiny_plain()
    h = _oracle_hg(inst)
    g = H.hg_load_csr(inst.n, inst.eptr, inst.pins, inst.c, inst.w, k_max=2)
    L = H.hg_max_block_weight(g, 2, inst.eps)
    part_o, stats_o, km_o = O.refine(h, 2, L, 5, inst.part)
    st = H.State(g, 2, inst.part)
    stats = torch.zeros(5 * H.STATS_WORDS, dtype=torch.int64, device="cuda")
    H.hg_refine(g, st, inst.eps, 5, stats)
    torch.cuda.synchronize()
    assert np.array_equal(st.part.cpu().numpy(), part_o)
    assert int(st.km1.item()) == km_o
    got = H.stats_to_dicts(stats)
    for r in range(5):
        got[r].pop("km1_delta_recomputed")
        assert got[r] == stats_o[r]


def test_golden_examples_on_gpu(H):
    """The hand-derived examples, run through the C ABI."""
    import json
    import os
    import torch
    path = os.path.join(os.path.dirname(__file__), "golden", "hand_examples.json")
    for ex in json.load(open(path))["examples"]:
        nets = ex["nets"]
        eptr = np.zeros(len(nets) + 1, np.int64)
        eptr[1:] = np.cumsum([len(x) for x in nets])
        pins = np.array([v for x in nets for v in x], np.int32)
        k = ex["k"]
        g = H.hg_load_csr(ex["n"], eptr, pins, np.array(ex["c"]), np.array(ex["w"]), k_max=k)
        assert H.hg_max_block_weight(g, k, ex["eps"]) == ex["lmax"]
        st = H.State(g, k, np.array(ex["part"], np.int32))
        H.hg_compute_pincounts(g, st)
        gains, _ = H.hg_gains(g, k, st.part, st.netstate)
        torch.cuda.synchronize()
        assert st.phi.view(-1, k).cpu().tolist() == ex["phi"]
        assert int(st.km1.item()) == ex["km1"]
        assert gains.view(-1, k).cpu().tolist() == ex["gains"]
        stats = torch.zeros(H.STATS_WORDS, dtype=torch.int64, device="cuda")
        for rnd in ex["rounds"]:
            H.hg_lp_round(g, st, ex["lmax"], stats)
            torch.cuda.synchronize()
            assert st.part.cpu().tolist() == rnd["part_after"], ex["name"]
            sg = H.stats_to_dicts(stats)[0]
            sg.pop("km1_delta_recomputed")
            assert sg == rnd["stats"], ex["name"]


def test_determinism_repeat(H):
    """Same inputs twice: bit-identical incidence, state and moves."""
    import torch
    inst = synth.random_power_law(5, 30000, 28000, 32, hi=40, unit=False, rounds=3)
    outs = []
    for _ in range(2):
        g = H.hg_load_csr(inst.n, inst.eptr, inst.pins, inst.c, inst.w, k_max=32)
        st = H.State(g, 32, inst.part)
        stats = torch.zeros(3 * H.STATS_WORDS, dtype=torch.int64, device="cuda")
        H.hg_refine(g, st, inst.eps, 3, stats, use_graph=False)
        torch.cuda.synchronize()
        outs.append([g.vnets.cpu().numpy(), st.part.cpu().numpy(), st.phi.cpu().numpy(),
                     st.netstate.cpu().numpy(), stats.cpu().numpy()])
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("nets,bad_at,bad", [
    (2, 3, -1),                   # negative pin, one tile
    (30000, 59999, 60000),        # pin = n in the last of 15 tiles
    (30000, 12345, -7),           # negative pin in a middle tile
    ((1 << 23) + 3, -1, 1 << 30),  # 2^24 + 6 pins: the long-sort tiles
])
def test_pin_range_check(H, nets, bad_at, bad):
    """The pins' range check rides on the first radix pass's digit count:
    a single bad pin anywhere, in either tile size, rejects the load."""
    eptr = np.arange(0, 2 * nets + 1, 2, dtype=np.int64)
    n = 2 * nets
    pins = np.arange(n, dtype=np.int32)
    good = pins[bad_at]
    pins[bad_at] = bad
    with pytest.raises(H.HgError) as ei:
        H.hg_load_csr(n, eptr, pins, k_max=2)
    assert ei.value.code == H.HG_ERR_INVALID
    assert "outside [0, n)" in str(ei.value)
    pins[bad_at] = good                               # the same load, valid: accepted
    g = H.hg_load_csr(n, eptr, pins, k_max=2)
    g.free()


def test_invalid_inputs_raise(H):
    import torch
    eptr = np.array([0, 2, 4], np.int64)
    with pytest.raises(H.HgError) as ei:                      # pin out of range
        H.hg_load_csr(3, eptr, np.array([0, 1, 1, 3], np.int32), k_max=2)
    assert ei.value.code == H.HG_ERR_INVALID
    with pytest.raises(H.HgError) as ei:                      # duplicate pin in a net
        H.hg_load_csr(3, eptr, np.array([0, 0, 1, 2], np.int32), k_max=2)
    assert ei.value.code == H.HG_ERR_INVALID
    with pytest.raises(H.HgError) as ei:                      # empty net
        H.hg_load_csr(3, np.array([0, 2, 2, 4], np.int64), np.array([0, 1, 1, 2], np.int32),
                      k_max=2)
    assert ei.value.code == H.HG_ERR_INVALID
    with pytest.raises(H.HgError) as ei:                      # zero weight
        H.hg_load_csr(3, eptr, np.array([0, 1, 1, 2], np.int32), vwgt=np.array([1, 0, 1]),
                      k_max=2)
    assert ei.value.code == H.HG_ERR_INVALID
    with pytest.raises(H.HgError) as ei:                      # net weight sum >= 2^31
        H.hg_load_csr(3, eptr, np.array([0, 1, 1, 2], np.int32),
                      ewgt=np.array([2 ** 30, 2 ** 30]), k_max=2)
    assert ei.value.code == H.HG_ERR_UNSUPPORTED
    g = H.hg_load_csr(3, eptr, np.array([0, 1, 1, 2], np.int32), k_max=4)
    with pytest.raises(H.HgError) as ei:                      # k beyond the workspace
        H.State(g, 8, np.zeros(3, np.int32))
        H.hg_compute_pincounts(g, H.State(g, 8, np.zeros(3, np.int32)))
    assert ei.value.code == H.HG_ERR_WORKSPACE
    ok = H.State(g, 2, np.array([0, 1, 1], np.int32))
    H.hg_compute_pincounts(g, ok)
    buf = torch.zeros(3 * 2 + 1, dtype=torch.int64, device="cuda")
    with pytest.raises(H.HgError) as ei:                      # gains not 16-byte aligned
        H.hg_gains(g, 2, ok.part, ok.netstate, gains=buf[1:])
    assert ei.value.code == H.HG_ERR_INVALID
    assert "aligned" in str(ei.value)
    st = H.State(g, 2, np.array([0, 5, 1], np.int32))         # partition id out of range
    H.hg_compute_pincounts(g, st)
    with pytest.raises(H.HgError) as ei:
        H.hg_sync_status(g)
    assert ei.value.code == H.HG_ERR_INVALID
    torch.cuda.synchronize()


@pytest.mark.parametrize("k", [8, 64])
def test_pincounts_and_rounds_with_unaligned_phi(H, k):
    """Phi rows are written with 16-byte stores only when the buffer is
    16-byte aligned; a buffer 4 bytes off takes the scalar path and must give
    the same state and rounds."""
    import torch
    inst = synth.random_power_law(60 + k, 7000, 6500, k, hi=20, unit=False, rounds=3)
    h = _oracle_hg(inst)
    g = H.hg_load_csr(inst.n, inst.eptr, inst.pins, inst.c, inst.w, k_max=k)
    sizes = H.state_sizes(g.n, g.m, k)
    views = {f: torch.empty(cnt, dtype=dt, device="cuda") for f, (dt, cnt) in sizes.items()}
    big = torch.empty(g.m * k + 4, dtype=torch.int32, device="cuda")
    views["phi"] = big[1:1 + g.m * k]
    assert views["phi"].data_ptr() % 16 == 4
    st = H.State(g, k, inst.part, views=views)
    H.hg_compute_pincounts(g, st)
    torch.cuda.synchronize()
    _check_state(H, g, st, h, k, inst.part)
    L = H.hg_max_block_weight(g, k, inst.eps)
    stats = torch.zeros(H.STATS_WORDS, dtype=torch.int64, device="cuda")
    part_o, elig_o = inst.part.copy(), np.ones(inst.n, np.uint8)
    for r in range(2):
        H.hg_lp_round(g, st, L, stats)
        torch.cuda.synchronize()
        part_o, elig_o, _, st_o = O.lp_round(h, k, L, part_o, elig_o)
        assert np.array_equal(st.part.cpu().numpy(), part_o), (k, r)
        _check_state(H, g, st, h, k, part_o)
    H.hg_sync_status(g)
