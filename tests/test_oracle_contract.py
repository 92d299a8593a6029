"""Pins of the oracle's contraction (section "Coarsening", subsection
"Contraction"):

* a hand-worked example (tests/golden/contract_examples.*);
* a brute-force contraction with Python sets and dicts on random tiny
  instances;
* km1 is preserved: for random partitions of the coarse hypergraph, km1 of
  the coarse partition equals km1 of its projection to the fine vertices
  (brute-force km1 on both sides); vertex weight is preserved;
* structure: coarse nets have >= 2 distinct increasing pins, no two are
  equal; identity clusterings only merge identical nets; one cluster leaves
  no net; bad ids and overweight clusters are refused.
"""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from tests import brute

from .test_oracle_pins import _hg, _random_tiny

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "contract_examples.json")


def _nets_of(h):
    return [list(h.pins[h.eptr[e]:h.eptr[e + 1]]) for e in range(h.m)]


def _brute_contract(nets, n, c, w, cluster):
    ids = sorted(set(int(x) for x in cluster))
    rank = {cid: r for r, cid in enumerate(ids)}
    mp = [rank[int(cluster[v])] for v in range(n)]
    cv = [0] * len(ids)
    for v in range(n):
        cv[mp[v]] += int(c[v])
    first = {}
    for e, net in enumerate(nets):
        s = frozenset(mp[v] for v in net)
        if len(s) < 2:
            continue
        if s not in first:
            first[s] = [e, 0]
        first[s][1] += int(w[e])
    kept = sorted(first.items(), key=lambda kv: kv[1][0])
    cn = [sorted(s) for s, _ in kept]
    cw = [v[1] for _, v in kept]
    return mp, cv, cn, cw


def test_hand_worked_contraction():
    with open(GOLDEN) as f:
        for ex in json.load(f)["examples"]:
            h = _hg(ex["nets"], ex["n"], np.array(ex["c"], np.int32), np.array(ex["w"], np.int32))
            mp, hc = O.contract(h, ex["cluster"])
            assert mp.tolist() == ex["map"]
            assert hc.c.tolist() == ex["cvwgt"]
            assert hc.eptr.tolist() == ex["ceptr"]
            assert hc.pins.tolist() == ex["cpins"]
            assert hc.w.tolist() == ex["cewgt"]
            cp = ex["coarse_part"]
            assert brute.km1(_nets_of(hc), hc.w, cp) == ex["km1"]
            assert brute.km1(ex["nets"], ex["w"], [cp[x] for x in mp]) == ex["km1"]


def _random_clustering(rng, n):
    kind = int(rng.integers(0, 3))
    if kind == 0:                                  # few big clusters
        return rng.integers(0, max(1, n // 3), n).astype(np.int32)
    if kind == 1:                                  # sparse ids anywhere in [0, n)
        return rng.choice(n, size=n).astype(np.int32)
    return np.where(rng.random(n) < 0.5, np.arange(n), rng.integers(0, n, n)).astype(np.int32)


def test_matches_brute_force_and_preserves_km1():
    rng = np.random.default_rng(41)
    merged = 0
    for _ in range(400):
        nets, n, k, c, w, part = _random_tiny(rng)
        h = _hg(nets, n, c, w)
        cl = _random_clustering(rng, n)
        mp, hc = O.contract(h, cl)
        bmp, bcv, bcn, bcw = _brute_contract(nets, n, c, w, cl)
        assert mp.tolist() == bmp
        assert hc.c.tolist() == bcv
        assert [list(x) for x in _nets_of(hc)] == bcn
        assert hc.w.tolist() == bcw
        assert int(hc.c.sum()) == int(c.sum())
        merged += len(bcn) < sum(1 for net in nets if len({bmp[v] for v in net}) > 1)
        cnets = _nets_of(hc)
        for net in cnets:
            assert len(net) >= 2 and all(a < b for a, b in zip(net, net[1:]))
        assert len({tuple(x) for x in cnets}) == len(cnets)
        for _ in range(3):
            kk = int(rng.integers(2, 5))
            cp = rng.integers(0, kk, hc.n)
            assert brute.km1(cnets, hc.w, cp) == brute.km1(nets, w, [cp[x] for x in mp])
    assert merged > 50


def test_edge_cases():
    rng = np.random.default_rng(42)
    nets = [[0, 1], [1, 2], [0, 1], [2, 3, 4], [1, 0]]
    nets = [sorted(x) for x in nets]
    h = _hg(nets, 5, np.ones(5, np.int32), np.array([1, 2, 3, 4, 5], np.int32))
    mp, hc = O.contract(h, np.arange(5))            # identity: identical nets merge
    assert mp.tolist() == list(range(5))
    assert _nets_of(hc) == [[0, 1], [1, 2], [2, 3, 4]] and hc.w.tolist() == [9, 2, 4]
    mp, hc = O.contract(h, np.full(5, 3))           # one cluster: no net survives
    assert hc.n == 1 and hc.m == 0 and hc.P == 0 and hc.c.tolist() == [5]
    with pytest.raises(ValueError):
        O.contract(h, np.array([0, 1, 2, 3, 5]))
    big = _hg(nets, 5, np.full(5, 2**30, np.int32), np.ones(5, np.int32))
    with pytest.raises(OverflowError):
        O.contract(big, np.zeros(5))
    del rng
