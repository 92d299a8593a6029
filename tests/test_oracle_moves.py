"""Pins of the oracle's move-sequence functions (exact gains of an ordered
sequence, best balanced prefix, the monotone LP round).

Each is checked against something other than its own arithmetic:
* exact gains: km1 recomputed from scratch before and after every move of the
  sequence (set-based brute force, tests/brute.py);
* the paper's Lemma on out-/in-move indices (section "Parallel Gain
  Calculation", subsection "Parallel Gain Recalculation"), evaluated in plain
  Python from the sequence alone, gives the same gains;
* best prefix: every prefix enumerated, block weights recounted from the
  partition;
* monotone round: km1 never increases, the applied moves are a prefix of the
  plain round's approved moves in (gain desc, id asc) order, the km1 drop is
  the sum of the prefix's exact gains, and when no two approved movers share
  a net nothing is cut and the round equals the plain one.
"""
import numpy as np
import pytest

from oracle import oracle as O
from tests import brute

from .test_oracle_pins import _hg, _random_tiny


def _random_sequence(rng, n, part, k, t=None):
    t = int(rng.integers(1, n + 1)) if t is None else t
    mu = rng.permutation(n)[:t].astype(np.int32)
    mt = np.array([(part[u] + 1 + rng.integers(0, k - 1)) % k for u in mu], np.int32)
    return mu, mt


def _lemma_gains(nets, w, part, mu, mt, k):
    """Exact gains from the Lemma's conditions, computed from the sequence
    and the start pin counts only (no replay)."""
    t = len(mu)
    src = {int(u): int(part[u]) for u in mu}
    out_max, in_min, out_cnt = {}, {}, {}
    for j, (u, b) in enumerate(zip(mu, mt), start=1):
        a = src[int(u)]
        for e, net in enumerate(nets):
            if u not in net:
                continue
            out_max[(e, a)] = max(out_max.get((e, a), 0), j)
            in_min[(e, int(b))] = min(in_min.get((e, int(b)), 1 << 60), j)
            out_cnt[(e, a)] = out_cnt.get((e, a), 0) + 1
    g = []
    for j, (u, b) in enumerate(zip(mu, mt), start=1):
        a, b = src[int(u)], int(b)
        tot = 0
        for e, net in enumerate(nets):
            if u not in net:
                continue
            we = 1 if w is None else int(w[e])
            psi_a = brute.pin_count(net, part, a) - out_cnt.get((e, a), 0)
            psi_b = brute.pin_count(net, part, b) - out_cnt.get((e, b), 0)
            if psi_a == 0 and out_max.get((e, a), 0) == j and in_min.get((e, a), 1 << 60) > j:
                tot += we
            if psi_b == 0 and in_min.get((e, b), 1 << 60) == j and out_max.get((e, b), 0) < j:
                tot -= we
        g.append(tot)
    return np.array(g, np.int64)


def test_move_gains_are_km1_deltas_of_the_replay():
    rng = np.random.default_rng(11)
    for _ in range(300):
        nets, n, k, c, w, part = _random_tiny(rng)
        h = _hg(nets, n, c, w)
        mu, mt = _random_sequence(rng, n, part, k)
        g = O.move_gains(h, k, part, mu, mt)
        cur = list(int(x) for x in part)
        for j, (u, b) in enumerate(zip(mu, mt)):
            before = brute.km1(nets, w, cur)
            cur[int(u)] = int(b)
            assert g[j] == before - brute.km1(nets, w, cur)


def test_lemma_conditions_give_the_exact_gains():
    rng = np.random.default_rng(12)
    for _ in range(300):
        nets, n, k, c, w, part = _random_tiny(rng)
        h = _hg(nets, n, c, w)
        mu, mt = _random_sequence(rng, n, part, k)
        assert np.array_equal(O.move_gains(h, k, part, mu, mt),
                              _lemma_gains(nets, w, part, mu, mt, k))


def test_move_gains_reject_invalid_sequences():
    rng = np.random.default_rng(13)
    nets, n, k, c, w, part = _random_tiny(rng, n=8, m=6, k=3)
    h = _hg(nets, n, c, w)
    u = 2
    with pytest.raises(ValueError):                       # a vertex twice
        O.move_gains(h, k, part, [u, u], [(part[u] + 1) % k, (part[u] + 2) % k])
    with pytest.raises(ValueError):                       # target = own block
        O.move_gains(h, k, part, [u], [part[u]])
    with pytest.raises(ValueError):                       # target outside [0, k)
        O.move_gains(h, k, part, [u], [k])


def test_best_prefix_by_enumeration():
    rng = np.random.default_rng(14)
    for _ in range(300):
        nets, n, k, c, w, part = _random_tiny(rng)
        h = _hg(nets, n, c, w)
        mu, mt = _random_sequence(rng, n, part, k)
        g = O.move_gains(h, k, part, mu, mt)
        total = int(c.astype(np.int64).sum())
        lm = int(rng.integers(total // k, total + 1))
        want_len, want_gain = 0, 0
        cur = part.copy()
        for p in range(1, len(mu) + 1):
            cur[mu[p - 1]] = mt[p - 1]
            W = np.bincount(cur, weights=c, minlength=k)
            if W.max() <= lm and g[:p].sum() >= want_gain:
                want_len, want_gain = p, int(g[:p].sum())
        assert O.best_prefix(h, k, lm, part, mu, mt, g) == (want_len, want_gain)


def test_exact_round_is_monotone_prefix_of_plain_round():
    rng = np.random.default_rng(15)
    cut_seen = 0
    for _ in range(400):
        nets, n, k, c, w, part = _random_tiny(rng)
        h = _hg(nets, n, c, w)
        L = int(rng.integers(int(c.sum()) // k, int(c.sum()) + 1))
        elig = np.ones(n, np.uint8)
        p_plain, e_plain, mv_plain, st_plain = O.lp_round(h, k, L, part, elig)
        p_ex, e_ex, mv_ex, st_ex, napp = O.lp_round_exact(h, k, L, part, elig)
        assert napp == st_plain["approved"]
        # the moved vertices are a prefix of the approved ones in (gain desc, id asc)
        g_sel = {u: brute.move_gain(nets, w, part, u, int(p_plain[u]))
                 for u in range(n) if mv_plain[u]}
        order = sorted(g_sel, key=lambda u: (-g_sel[u], u))
        moved = [u for u in range(n) if mv_ex[u]]
        assert sorted(order[:len(moved)]) == moved
        for u in moved:
            assert p_ex[u] == p_plain[u]
        # km1 drop = sum of the exact gains of the prefix, never negative
        before = brute.km1(nets, w, part)
        assert st_ex["km1_after"] == brute.km1(nets, w, p_ex)
        assert st_ex["km1_delta"] == before - st_ex["km1_after"] >= 0
        mu = np.array(order, np.int32)
        mt = np.array([p_plain[u] for u in order], np.int32)
        gx = O.move_gains(h, k, part, mu, mt)
        assert st_ex["km1_delta"] == int(gx[:len(moved)].sum()) == max(
            [0] + list(np.cumsum(gx)))
        # never heavier than L_max where the plain round would not be
        W = np.bincount(p_ex, weights=c, minlength=k)
        W0 = np.bincount(part, weights=c, minlength=k)
        assert all(W[i] <= L or W[i] <= W0[i] for i in range(k))
        if len(moved) < napp:
            cut_seen += 1
        # disjoint movers: exact gains are the select gains, nothing is cut
        touched = [set(brute.incident(nets, u)) for u in order]
        if all(not (touched[i] & touched[j]) for i in range(len(order))
               for j in range(i)):
            assert len(moved) == napp
            assert np.array_equal(p_ex, p_plain)
    assert cut_seen > 0          # the instances exercise the prefix cut


def test_exact_refine_never_increases_km1():
    rng = np.random.default_rng(16)
    for _ in range(40):
        nets, n, k, c, w, part = _random_tiny(rng, n=12, m=14)
        h = _hg(nets, n, c, w)
        L = O.lmax(int(c.sum()), k, 0.2)
        _, stats, km = O.refine_exact(h, k, L, 4, part)
        prev = brute.km1(nets, w, part)
        for s in stats:
            assert s["km1_after"] <= prev
            prev = s["km1_after"]
        assert km == prev
