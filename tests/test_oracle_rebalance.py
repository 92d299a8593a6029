"""Pins of the oracle's rebalancing round (section "Rebalancing", read as a
synchronous deterministic round):

* hand-worked rounds (tests/golden/rebalance_examples.*);
* a brute-force round (tests/brute.py) whose gains are km1 differences of
  single moves, on random tiny instances with random L_max;
* invariants: only vertices of overloaded blocks move, no block that was
  within L_max leaves it, no overloaded block gets heavier, a balanced
  partition is a fixed point, each source sheds at most its excess plus one
  vertex; the driver is the rounds in a row.
"""
import json
import os

import numpy as np

from oracle import oracle as O
from tests import brute

from .test_oracle_pins import _hg, _random_tiny

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "rebalance_examples.json")


def test_hand_worked_rounds():
    with open(GOLDEN) as f:
        examples = json.load(f)["examples"]
    for ex in examples:
        c = np.array(ex["c"], np.int32)
        w = np.array(ex["w"], np.int32)
        h = _hg(ex["nets"], ex["n"], c, w)
        part = np.array(ex["part"], np.int32)
        elig = np.zeros(ex["n"], np.uint8)
        for r, want in enumerate(ex["rounds"]):
            part, elig, moved, st = O.rebalance_round(h, ex["k"], ex["lmax"], part, elig)
            assert part.tolist() == want["part"], (ex["name"], r)
            assert elig.tolist() == want["eligible"], (ex["name"], r)
            assert st == want["stats"], (ex["name"], r, st)
        # the driver gives the same
        p2, e2, stats, km = O.rebalance(h, ex["k"], ex["lmax"], len(ex["rounds"]), ex["part"])
        assert p2.tolist() == ex["rounds"][-1]["part"]
        assert [s for s in stats] == [x["stats"] for x in ex["rounds"]]
        assert km == ex["rounds"][-1]["stats"]["km1_after"]


def _tight_lmax(rng, c, k):
    total = int(c.sum())
    return int(rng.integers(max(1, total // k), total // k + 4))


def test_matches_brute_force():
    rng = np.random.default_rng(31)
    moved_rounds = 0
    for _ in range(400):
        nets, n, k, c, w, part = _random_tiny(rng)
        if rng.integers(0, 2):               # pile most vertices into one block
            part = np.where(rng.random(n) < 0.7, 0, part).astype(np.int32)
        h = _hg(nets, n, c, w)
        L = _tight_lmax(rng, c, k)
        elig = rng.integers(0, 2, n).astype(np.uint8)
        p_o, e_o, m_o, s_o = O.rebalance_round(h, k, L, part, elig)
        p_b, e_b, m_b, s_b = brute.rebalance_round(nets, n, c, w, k, L, part, elig)
        assert p_o.tolist() == p_b
        assert e_o.tolist() == e_b
        assert m_o.tolist() == m_b
        assert s_o == s_b
        moved_rounds += s_o["approved"] > 0
    assert moved_rounds > 100


def test_invariants():
    rng = np.random.default_rng(32)
    for _ in range(400):
        nets, n, k, c, w, part = _random_tiny(rng, n=int(rng.integers(4, 16)))
        part = np.where(rng.random(n) < 0.6, 0, part).astype(np.int32)
        h = _hg(nets, n, c, w)
        L = _tight_lmax(rng, c, k)
        W0 = np.bincount(part, weights=c, minlength=k).astype(np.int64)
        new, _, moved, st = O.rebalance_round(h, k, L, part, np.zeros(n, np.uint8))
        W1 = np.bincount(new, weights=c, minlength=k).astype(np.int64)
        over = W0 > L
        for u in range(n):
            if moved[u]:
                assert over[part[u]] and new[u] != part[u]
            else:
                assert new[u] == part[u]
        for i in range(k):
            if not over[i]:
                assert W1[i] <= L
            else:
                assert W1[i] <= W0[i]
                shed = W0[i] - W1[i]
                assert shed < W0[i] - L + int(c.max()) or shed == 0
        assert st["km1_after"] == brute.km1(nets, w, new)
        if not over.any():
            assert np.array_equal(new, part) and st["approved"] == 0


def test_driver_is_rounds_in_a_row():
    rng = np.random.default_rng(33)
    for _ in range(60):
        nets, n, k, c, w, part = _random_tiny(rng, n=12, m=12)
        part = np.where(rng.random(n) < 0.8, 0, part).astype(np.int32)
        h = _hg(nets, n, c, w)
        L = _tight_lmax(rng, c, k)
        p, e = part.copy(), np.zeros(n, np.uint8)
        want = []
        for _ in range(4):
            p, e, _, st = O.rebalance_round(h, k, L, p, e)
            want.append(st)
        p2, e2, stats, km = O.rebalance(h, k, L, 4, part)
        assert np.array_equal(p2, p) and np.array_equal(e2, e)
        assert stats == want
        assert km == brute.km1(nets, w, p)
        mx = [s["max_block_weight"] for s in stats]
        assert all(b <= a for a, b in zip(mx, mx[1:]))
