"""Pins of the CPU oracle against what the paper and mathematics fix.

Nothing here touches a GPU.  The oracle is checked against:
* hand-derived worked examples (tests/golden/hand_examples.*);
* a set-based brute force that computes gains as objective deltas
  (tests/brute.py), on many random tiny hypergraphs;
* closed forms and special cases: constant partition, graphs (all nets of
  size 2) where km1 is the edge cut, k = 2 where km1 is the cut-net weight,
  the upper bound sum (min(k,|e|)-1) w(e);
* invariants: Phi row sums, lambda as the nonzero count, balance after every
  round, attributed-gain total = recomputed km1 drop, no negative-gain move,
  the paper's gain-cache update rules after one move.
"""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from tests import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_examples.json")


def _csr(nets):
    eptr = np.zeros(len(nets) + 1, np.int64)
    eptr[1:] = np.cumsum([len(e) for e in nets])
    pins = np.array([v for e in nets for v in e], np.int32)
    return eptr, pins


def _random_tiny(rng, n=None, m=None, k=None, weighted=None):
    n = n or int(rng.integers(2, 13))
    m = m or int(rng.integers(1, 13))
    k = k or int(rng.integers(2, 5))
    weighted = bool(rng.integers(0, 2)) if weighted is None else weighted
    nets = []
    for _ in range(m):
        s = int(rng.integers(1, min(n, 5) + 1))
        nets.append(sorted(rng.choice(n, size=s, replace=False).tolist()))
    c = rng.integers(1, 5, n).astype(np.int32) if weighted else np.ones(n, np.int32)
    w = rng.integers(1, 5, m).astype(np.int32) if weighted else np.ones(m, np.int32)
    part = rng.integers(0, k, n).astype(np.int32)
    return nets, n, k, c, w, part


def _hg(nets, n, c, w):
    eptr, pins = _csr(nets)
    return O.Hypergraph(n, eptr, pins, c, w)


# ---------------------------------------------------------------- golden


def _golden():
    with open(GOLDEN) as f:
        return json.load(f)["examples"]


@pytest.mark.parametrize("ex", _golden(), ids=lambda e: e["name"])
def test_golden_hand_examples(ex):
    h = _hg(ex["nets"], ex["n"], np.array(ex["c"], np.int32), np.array(ex["w"], np.int32))
    k = ex["k"]
    assert O.check_hypergraph(h) == O.OR_OK
    L = O.lmax(O.total_vertex_weight(h), k, ex["eps"])
    assert L == ex["lmax"]
    phi = O.pin_counts(h, ex["part"], k)
    assert phi.tolist() == ex["phi"]
    lam, _ = O.connectivity(phi, k)
    assert lam.tolist() == ex["lambda"]
    assert O.km1(h, lam) == ex["km1"]
    g, b = O.gains(h, ex["part"], k)
    assert g.tolist() == ex["gains"]
    assert b.tolist() == ex["benefit"]
    part = np.array(ex["part"], np.int32)
    elig = np.ones(ex["n"], np.uint8)
    for rnd in ex["rounds"]:
        part, elig, moved, st = O.lp_round(h, k, L, part, elig)
        assert part.tolist() == rnd["part_after"]
        assert np.nonzero(moved)[0].tolist() == rnd["moved"]
        assert np.nonzero(elig)[0].tolist() == rnd["next_eligible"]
        assert st == rnd["stats"]


@pytest.mark.parametrize("ex", _golden(), ids=lambda e: e["name"])
def test_golden_brute_agrees(ex):
    """The brute force reproduces the hand derivation too (pins the pin)."""
    nets = ex["nets"]
    part = list(ex["part"])
    assert brute.km1(nets, ex["w"], part) == ex["km1"]
    for u in range(ex["n"]):
        for i in range(ex["k"]):
            assert brute.move_gain(nets, ex["w"], part, u, i) == ex["gains"][u][i]
    elig = [1] * ex["n"]
    for rnd in ex["rounds"]:
        part, elig, moved, st = brute.lp_round(nets, ex["n"], ex["c"], ex["w"], ex["k"],
                                               ex["lmax"], part, elig)
        assert part == rnd["part_after"]
        assert st == rnd["stats"]


# ---------------------------------------------------------------- definitions


def test_random_tiny_against_brute_force():
    rng = np.random.default_rng(12345)
    for _ in range(300):
        nets, n, k, c, w, part = _random_tiny(rng)
        h = _hg(nets, n, c, w)
        assert O.check_hypergraph(h) == O.OR_OK
        phi = O.pin_counts(h, part, k)
        for j, e in enumerate(nets):
            for i in range(k):
                assert phi[j, i] == brute.pin_count(e, part, i)
        lam, conn = O.connectivity(phi, k)
        for j, e in enumerate(nets):
            blocks = brute.blocks_of(e, part)
            assert lam[j] == len(blocks)
            assert {i for i in range(k) if conn[j, i // 32] >> (i % 32) & 1} == blocks
        assert O.km1(h, lam) == brute.km1(nets, w, part)
        g, b = O.gains(h, part, k)
        for u in range(n):
            for i in range(k):
                assert g[u, i] == brute.move_gain(nets, w, part, u, i), (u, i)
        W = O.block_weights(h, part, k)
        for i in range(k):
            assert W[i] == brute.block_weight(part, c, i)


def test_lp_round_against_brute_force():
    rng = np.random.default_rng(777)
    for trial in range(300):
        nets, n, k, c, w, part = _random_tiny(rng)
        h = _hg(nets, n, c, w)
        total = int(c.sum())
        eps = float(rng.choice([0.03, 0.1, 0.3, 0.6]))
        L = O.lmax(total, k, eps)
        elig = (rng.random(n) < 0.8).astype(np.uint8) if trial % 3 else np.ones(n, np.uint8)
        p_o, e_o, m_o, s_o = O.lp_round(h, k, L, part, elig)
        p_b, e_b, m_b, s_b = brute.lp_round(nets, n, c, w, k, L, part, elig)
        assert p_o.tolist() == p_b
        assert e_o.tolist() == e_b
        assert m_o.tolist() == m_b
        assert s_o == s_b, (trial, s_o, s_b)


# ---------------------------------------------------------------- special cases


def test_constant_partition_has_zero_km1_and_no_boundary():
    rng = np.random.default_rng(5)
    nets, n, k, c, w, _ = _random_tiny(rng, n=10, m=10, k=3)
    h = _hg(nets, n, c, w)
    part = np.full(n, 2, np.int32)
    lam, _ = O.connectivity(O.pin_counts(h, part, k), k)
    assert O.km1(h, lam) == 0
    _, _, moved, st = O.lp_round(h, k, 10 ** 9, part, np.ones(n, np.uint8))
    assert st["boundary"] == 0 and st["approved"] == 0 and moved.sum() == 0


def test_graph_km1_is_weighted_edge_cut():
    """All nets of size 2: km1 is the weighted edge cut of the graph."""
    rng = np.random.default_rng(6)
    n, k = 40, 4
    edges = set()
    while len(edges) < 120:
        a, b = sorted(rng.choice(n, 2, replace=False).tolist())
        edges.add((a, b))
    edges = sorted(edges)
    w = rng.integers(1, 10, len(edges)).astype(np.int32)
    part = rng.integers(0, k, n).astype(np.int32)
    h = _hg([list(e) for e in edges], n, None, w)
    lam, _ = O.connectivity(O.pin_counts(h, part, k), k)
    cut = sum(int(w[j]) for j, (a, b) in enumerate(edges) if part[a] != part[b])
    assert O.km1(h, lam) == cut


def test_bipartition_km1_is_cut_net_weight_and_fm_gain():
    """k = 2: km1 = weight of cut nets, and the gain is the classical FM gain
    (nets where u is alone on its side minus nets entirely on u's side)."""
    rng = np.random.default_rng(7)
    for _ in range(50):
        nets, n, _, c, w, _ = _random_tiny(rng, k=2)
        part = rng.integers(0, 2, n).astype(np.int32)
        h = _hg(nets, n, c, w)
        lam, _ = O.connectivity(O.pin_counts(h, part, 2), 2)
        cut = sum(int(w[j]) for j, e in enumerate(nets) if len({int(part[v]) for v in e}) == 2)
        assert O.km1(h, lam) == cut
        g, _ = O.gains(h, part, 2)
        for u in range(n):
            a = int(part[u])
            inc = [j for j, e in enumerate(nets) if u in e]
            from_side = sum(int(w[j]) for j in inc
                            if sum(1 for v in nets[j] if part[v] == a) == 1)
            to_side_empty = sum(int(w[j]) for j in inc
                                if all(part[v] == a for v in nets[j]))
            assert g[u, 1 - a] == from_side - to_side_empty


def test_km1_upper_bound_and_phi_invariants():
    rng = np.random.default_rng(8)
    for _ in range(100):
        nets, n, k, c, w, part = _random_tiny(rng)
        h = _hg(nets, n, c, w)
        phi = O.pin_counts(h, part, k)
        lam, _ = O.connectivity(phi, k)
        sizes = np.array([len(e) for e in nets])
        assert (phi.sum(axis=1) == sizes).all()
        assert (phi >= 0).all() and (phi <= sizes[:, None]).all()
        assert (lam == (phi > 0).sum(axis=1)).all()
        assert (lam >= 1).all() and (lam <= np.minimum(k, sizes)).all()
        bound = sum((min(k, len(e)) - 1) * int(w[j]) for j, e in enumerate(nets))
        assert 0 <= O.km1(h, lam) <= bound


def test_gain_cache_update_rules_after_one_move():
    """Section "Gain Caching": after moving u from V_a to V_b, the four update
    rules applied to b(.) and p_.(.) of the other vertices give exactly the
    b and p recomputed from scratch on the new partition."""
    rng = np.random.default_rng(9)
    for _ in range(200):
        nets, n, k, c, w, part = _random_tiny(rng)
        h = _hg(nets, n, c, w)
        u = int(rng.integers(0, n))
        a = int(part[u])
        bb = int((a + 1 + rng.integers(0, k - 1)) % k)
        g0, b0 = O.gains(h, part, k)
        p0 = b0[:, None] - g0                      # p_i(v) = b(v) - g_i(v), i != Pi(v)
        new = part.copy()
        new[u] = bb
        phi1 = O.pin_counts(h, new, k)
        g1, b1 = O.gains(h, new, k)
        p1 = b1[:, None] - g1
        b_pred = b0.copy()
        p_pred = p0.copy()
        for j, e in enumerate(nets):
            if u not in e:
                continue
            we = int(w[j])
            if phi1[j, a] == 0:
                for v in e:
                    p_pred[v, a] += we
            if phi1[j, a] == 1:
                for v in e:
                    if new[v] == a:
                        b_pred[v] += we
            if phi1[j, bb] == 1:
                for v in e:
                    p_pred[v, bb] -= we
            if phi1[j, bb] == 2:
                for v in e:
                    if new[v] == bb:
                        b_pred[v] -= we
        for v in range(n):
            if v == u:
                continue                            # b(u) is recomputed after moves
            assert b_pred[v] == b1[v]
            for i in range(k):
                if i != new[v] and i != part[v]:
                    assert p_pred[v, i] == p1[v, i], (v, i)


# ---------------------------------------------------------------- LP invariants


def test_lp_invariants_on_random_instances():
    """Balance is never violated from a balanced start, overloaded blocks never
    gain weight, the recomputed km1 drop is reported, candidates never have a
    negative gain, and approval is a maximal prefix."""
    rng = np.random.default_rng(10)
    import synth
    for trial in range(6):
        inst = synth.random_power_law(100 + trial, 300, 280, int(rng.choice([2, 3, 5, 8])),
                                      hi=12, unit=bool(trial % 2))
        h = O.Hypergraph(inst.n, inst.eptr, inst.pins, inst.c, inst.w)
        L = O.lmax(O.total_vertex_weight(h), inst.k, inst.eps)
        part = inst.part.copy()
        elig = np.ones(inst.n, np.uint8)
        for r in range(6):
            W0 = O.block_weights(h, part, inst.k)
            g, _ = O.gains(h, part, inst.k)
            lam0, _ = O.connectivity(O.pin_counts(h, part, inst.k), inst.k)
            km0 = O.km1(h, lam0)
            new, elig, moved, st = O.lp_round(h, inst.k, L, part, elig)
            W1 = O.block_weights(h, new, inst.k)
            for i in range(inst.k):
                if W0[i] <= L:
                    assert W1[i] <= L
                else:
                    assert W1[i] <= W0[i]
            lam1, _ = O.connectivity(O.pin_counts(h, new, inst.k), inst.k)
            assert st["km1_delta"] == km0 - O.km1(h, lam1)
            for u in np.nonzero(moved)[0]:
                assert g[u, new[u]] >= 0
            part = new


def test_disjoint_movers_delta_equals_sum_of_gains():
    """When no two approved movers share a net, the round's km1 drop is the sum
    of their individual gains (each gain is an exact objective delta)."""
    rng = np.random.default_rng(11)
    hits = 0
    for _ in range(400):
        nets, n, k, c, w, part = _random_tiny(rng)
        h = _hg(nets, n, c, w)
        L = O.lmax(int(c.sum()), k, 0.6)
        g, _ = O.gains(h, part, k)
        new, _, moved, st = O.lp_round(h, k, L, part, np.ones(n, np.uint8))
        movers = np.nonzero(moved)[0].tolist()
        shared = any(sum(1 for v in e if moved[v]) > 1 for e in nets)
        if movers and not shared:
            hits += 1
            assert st["km1_delta"] == sum(int(g[u, new[u]]) for u in movers)
    assert hits > 20


def test_lmax_formula():
    assert O.lmax(10_000, 2, 0.03) == 5150
    assert O.lmax(10_001, 2, 0.03) == 5151        # ceil(10001/2) = 5001 -> 5151.03
    assert O.lmax(8, 3, 0.5) == 4
    assert O.lmax(100, 7, 0.03) == 15             # ceil = 15, 15.45 -> 15


def test_refine_records_empty_rounds_after_convergence():
    ex = _golden()[0]
    h = _hg(ex["nets"], ex["n"], np.array(ex["c"], np.int32), np.array(ex["w"], np.int32))
    part, stats, km = O.refine(h, ex["k"], ex["lmax"], 5, ex["part"])
    assert km == 2
    assert stats[0] == ex["rounds"][0]["stats"]
    for s in stats[2:]:
        assert s["eligible"] == 0 and s["approved"] == 0 and s["km1_after"] == 2


def test_check_rejects_invalid_inputs():
    h = _hg([[0, 1], [1, 1]], 3, None, None)      # duplicate pin
    assert O.check_hypergraph(h) == O.OR_ERR_INVALID
    h = _hg([[0, 3]], 3, None, None)              # pin out of range
    assert O.check_hypergraph(h) == O.OR_ERR_INVALID
    eptr = np.array([0, 2, 2], np.int64)          # empty net
    h = O.Hypergraph(3, eptr, np.array([0, 1], np.int32))
    assert O.check_hypergraph(h) == O.OR_ERR_INVALID
    h = _hg([[0, 1]], 2, np.array([1, 0], np.int32), None)   # zero weight
    assert O.check_hypergraph(h) == O.OR_ERR_INVALID
    h = _hg([[0, 1]], 2, None, None)
    assert O.check_partition(h, np.array([0, 2], np.int32), 2) == O.OR_ERR_INVALID
