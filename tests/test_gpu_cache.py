"""GPU parity of the gain cache, through the C ABI: the initial cache equals
the oracle's cache of the partition, every cached round makes exactly the
plain round's moves (all state and the round record bit-identical), and
after each round the cache equals the oracle's cache of the new partition.
"""
import numpy as np
import pytest

import synth
from oracle import oracle as O

from .test_gpu_parity import _hub_instance, _oracle_hg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2010_10272_amd import hgref
    return hgref


def _instances():
    yield "plaw-k2-u", lambda: synth.random_power_law(301, 9000, 8500, 2, hi=24, rounds=4)
    yield "plaw-k7-w", lambda: synth.random_power_law(302, 7000, 6600, 7, hi=16, unit=False,
                                                      rounds=4)
    yield "plaw-k64-u", lambda: synth.random_power_law(303, 8000, 7800, 64, hi=24, rounds=4)
    yield "plaw-k200-w", lambda: synth.random_power_law(304, 6000, 5600, 200, hi=12,
                                                        unit=False, rounds=3)
    yield "plaw-k256-u", lambda: synth.random_power_law(305, 5000, 5200, 256, hi=10, rounds=3)
    yield "band-k16", lambda: synth.sparse_matrix(16, seed=305, rows=30000, cols=30000,
                                                  band=1000, rounds=4)
    yield "hub-k16-w", lambda: _hub_instance(8, 6000, 5000, 16, 400, True)
    yield "hub-k3-u", lambda: _hub_instance(9, 5000, 4000, 3, 600, False)


INSTANCES = list(_instances())


def _check_cache(H, g, k, cache, h, part, what):
    b, wi, p = H.cache_views(g, k, cache)
    wb, wwi, wp = O.gain_cache(h, part, k)
    assert np.array_equal(b.cpu().numpy().astype(np.int64), wb), what
    assert np.array_equal(wi.cpu().numpy().astype(np.int64), wwi), what
    assert np.array_equal(p.cpu().numpy().astype(np.int64), wp), what


@pytest.mark.parametrize("name,make", INSTANCES, ids=[c[0] for c in INSTANCES])
def test_cached_rounds_equal_plain_rounds(H, name, make):
    import torch
    inst = make()
    h = _oracle_hg(inst)
    k = inst.k
    g = H.hg_load_csr(inst.n, inst.eptr, inst.pins, inst.c, inst.w, k_max=k)
    L = H.hg_max_block_weight(g, k, inst.eps)
    a = H.State(g, k, inst.part)          # plain rounds
    b = H.State(g, k, inst.part)          # cached rounds
    H.hg_compute_pincounts(g, a)
    H.hg_compute_pincounts(g, b)
    cache = H.gain_cache(g, k)
    cache.fill_(-7)                       # nothing may read what init does not write
    H.hg_gain_cache_init(g, k, b.part, b.netstate, cache)
    torch.cuda.synchronize()
    _check_cache(H, g, k, cache, h, inst.part, (name, "init"))
    sa = torch.zeros(H.STATS_WORDS, dtype=torch.int64, device="cuda")
    sb = torch.zeros(H.STATS_WORDS, dtype=torch.int64, device="cuda")
    moved_any = 0
    for r in range(inst.rounds + 2):
        H.hg_lp_round(g, a, L, sa)
        H.hg_lp_round_cached(g, b, L, sb, cache)
        torch.cuda.synchronize()
        assert torch.equal(sa, sb), (name, r, H.stats_to_dicts(sa), H.stats_to_dicts(sb))
        for f in H.STATE_FIELDS:
            assert torch.equal(getattr(a, f), getattr(b, f)), (name, r, f)
        part = b.part.cpu().numpy()
        _check_cache(H, g, k, cache, h, part, (name, r))
        moved_any += int(b.moved.sum().item())
    H.hg_sync_status(g)
    assert moved_any > 0


@pytest.mark.parametrize("name,make", INSTANCES[1:3] + INSTANCES[6:7],
                         ids=[c[0] for c in INSTANCES[1:3] + INSTANCES[6:7]])
def test_refine_cached_matches_oracle(H, name, make):
    import torch
    inst = make()
    h = _oracle_hg(inst)
    k = inst.k
    g = H.hg_load_csr(inst.n, inst.eptr, inst.pins, inst.c, inst.w, k_max=k)
    L = H.hg_max_block_weight(g, k, inst.eps)
    part_o, stats_o, km_o = O.refine(h, k, L, inst.rounds, inst.part)
    st = H.State(g, k, inst.part)
    cache = H.gain_cache(g, k)
    stats = torch.zeros(inst.rounds * H.STATS_WORDS, dtype=torch.int64, device="cuda")
    for rep in range(2):                  # the second run starts over from the same part
        st.part.copy_(torch.as_tensor(inst.part))
        H.hg_refine_cached(g, st, inst.eps, inst.rounds, stats, cache)
        torch.cuda.synchronize()
        assert np.array_equal(st.part.cpu().numpy(), part_o), (name, rep)
        got = H.stats_to_dicts(stats)
        for r in range(inst.rounds):
            assert got[r].pop("km1_delta_recomputed") == got[r]["km1_delta"]
            assert got[r] == stats_o[r], (name, rep, r)
        assert int(st.km1.item()) == km_o
        _check_cache(H, g, k, cache, h, part_o, (name, rep))
    H.hg_sync_status(g)


def test_cache_arguments_are_checked(H):
    import torch
    inst = synth.random_power_law(306, 500, 400, 4, hi=8, rounds=1)
    g = H.hg_load_csr(inst.n, inst.eptr, inst.pins, inst.c, inst.w, k_max=4)
    st = H.State(g, 4, inst.part)
    H.hg_compute_pincounts(g, st)
    cache = H.gain_cache(g, 4)
    stats = torch.zeros(H.STATS_WORDS, dtype=torch.int64, device="cuda")
    assert H._lib.hg_gain_cache_bytes(0, 4) == -1
    assert H._lib.hg_gain_cache_bytes(10, 1) == -1
    with pytest.raises(H.HgError):        # misaligned cache
        H.hg_gain_cache_init(g, 4, st.part, st.netstate, cache[1:])
    st.moved = None
    with pytest.raises((H.HgError, AttributeError, TypeError)):
        H.hg_lp_round_cached(g, st, 10**6, stats, cache)
    torch.cuda.synchronize()
