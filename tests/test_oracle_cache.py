"""Pins of the oracle's gain cache (subsection "Gain Caching": b(u) and the
penalties p_i(u) stored apart, updated as vertices move).

* b, w(I) and p by the set-based definitions (tests/brute.py), and
  b(u) - p_i(u) equal to the km1 delta of moving u to block i;
* the paper's four per-move update rules, applied move by move in any order
  (with b recomputed for the moved vertices afterwards), reach the cache of
  the final partition;
* the per-net aggregate of those rules over a whole synchronous round (the
  form the GPU finalize applies: p_i(v) changes where block i entered or left
  Lambda(e), b(v) of a vertex that stayed where its block entered or left
  the set of blocks holding exactly one pin of e) reaches it too.
"""
import numpy as np

from oracle import oracle as O
from tests import brute

from .test_oracle_pins import _hg, _random_tiny


def test_gain_cache_by_definition():
    rng = np.random.default_rng(21)
    for _ in range(300):
        nets, n, k, c, w, part = _random_tiny(rng)
        h = _hg(nets, n, c, w)
        b, wi, p = O.gain_cache(h, part, k)
        for u in range(n):
            inc = brute.incident(nets, u)
            a = int(part[u])
            assert wi[u] == sum(int(w[e]) for e in inc)
            assert b[u] == sum(int(w[e]) for e in inc if brute.pin_count(nets[e], part, a) == 1)
            for i in range(k):
                assert p[u, i] == sum(int(w[e]) for e in inc
                                      if brute.pin_count(nets[e], part, i) == 0)
                if i != a:
                    assert b[u] - p[u, i] == brute.move_gain(nets, w, part, u, i)
            assert p[u, a] == 0


def _moves(rng, n, k, part):
    t = int(rng.integers(1, n + 1))
    mu = rng.permutation(n)[:t]
    return {int(u): int((part[u] + 1 + rng.integers(0, k - 1)) % k) for u in mu}


def test_four_rules_move_by_move_reach_the_final_cache():
    rng = np.random.default_rng(22)
    for _ in range(300):
        nets, n, k, c, w, part = _random_tiny(rng)
        h = _hg(nets, n, c, w)
        b, _, p = O.gain_cache(h, part, k)
        b = b.copy()
        p = p.copy()
        cur = part.copy()
        phi = [[brute.pin_count(e, cur, i) for i in range(k)] for e in nets]
        moves = _moves(rng, n, k, part)
        for u in rng.permutation(sorted(moves)):
            u = int(u)
            src, dst = int(cur[u]), moves[u]
            cur[u] = dst
            for e in brute.incident(nets, u):
                we = int(w[e])
                phi[e][src] -= 1
                phi[e][dst] += 1
                if phi[e][src] == 0:
                    for v in nets[e]:
                        p[v, src] += we
                if phi[e][src] == 1:
                    for v in nets[e]:
                        if cur[v] == src:
                            b[v] += we
                if phi[e][dst] == 1:
                    for v in nets[e]:
                        p[v, dst] -= we
                if phi[e][dst] == 2:
                    for v in nets[e]:
                        if cur[v] == dst:
                            b[v] -= we
        want_b, _, want_p = O.gain_cache(h, cur, k)
        assert np.array_equal(p, want_p)
        for v in range(n):
            if v in moves:            # b of a moved vertex is stale until recomputed
                b[v] = want_b[v]
        assert np.array_equal(b, want_b)


def test_round_aggregate_reaches_the_final_cache():
    rng = np.random.default_rng(23)
    rounds_with_moves = 0
    for _ in range(300):
        nets, n, k, c, w, part = _random_tiny(rng)
        h = _hg(nets, n, c, w)
        b, _, p = O.gain_cache(h, part, k)
        b = b.copy()
        p = p.copy()
        if rng.integers(0, 2):
            L = int(rng.integers(int(c.sum()) // k, int(c.sum()) + 1))
            new, _, moved, _ = O.lp_round(h, k, L, part, np.ones(n, np.uint8))
        else:
            mv = _moves(rng, n, k, part)
            new = part.copy()
            for u, t in mv.items():
                new[u] = t
            moved = (new != part).astype(np.uint8)
        rounds_with_moves += bool(moved.any())
        for e, net in enumerate(nets):
            if not any(moved[v] for v in net):
                continue
            we = int(w[e])
            lam_old = {i for i in range(k) if brute.pin_count(net, part, i) > 0}
            lam_new = {i for i in range(k) if brute.pin_count(net, new, i) > 0}
            one_old = {i for i in range(k) if brute.pin_count(net, part, i) == 1}
            one_new = {i for i in range(k) if brute.pin_count(net, new, i) == 1}
            for v in net:
                for i in lam_old ^ lam_new:
                    p[v, i] += we if i in lam_old else -we
                cv = int(new[v])
                if not moved[v] and cv in one_old ^ one_new:
                    b[v] += we if cv in one_new else -we
        want_b, _, want_p = O.gain_cache(h, new, k)
        assert np.array_equal(p, want_p)
        for v in range(n):
            if moved[v]:
                b[v] = sum(int(w[e]) for e in brute.incident(nets, v)
                           if brute.pin_count(nets[e], new, int(new[v])) == 1)
        assert np.array_equal(b, want_b)
    assert rounds_with_moves > 100
