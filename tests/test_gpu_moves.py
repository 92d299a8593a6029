"""GPU parity of the move-sequence calls (exact gains of an ordered sequence,
best balanced prefix) and of the monotone label-propagation round, through
the C ABI, against the oracle.  Everything is integer: exact equality.
"""
import numpy as np
import pytest

import synth
from oracle import oracle as O

from .test_gpu_parity import _check_state, _hub_instance, _oracle_hg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2010_10272_amd import hgref
    return hgref


def _instances():
    yield "plaw-k2-u", lambda: synth.random_power_law(201, 9000, 8500, 2, hi=24, rounds=4)
    yield "plaw-k7-w", lambda: synth.random_power_law(202, 7000, 6600, 7, hi=16, unit=False,
                                                      rounds=4)
    yield "plaw-k64-u", lambda: synth.random_power_law(203, 8000, 7800, 64, hi=24, rounds=4)
    yield "plaw-k200-w", lambda: synth.random_power_law(204, 6000, 5600, 200, hi=12,
                                                        unit=False, rounds=3)
    yield "band-k16", lambda: synth.sparse_matrix(16, seed=205, rows=30000, cols=30000,
                                                  band=1000, rounds=4)
    yield "hub-k16-w", lambda: _hub_instance(8, 6000, 5000, 16, 400, True)


INSTANCES = list(_instances())


def _sequence(rng, inst, t):
    mu = rng.permutation(inst.n)[:t].astype(np.int32)
    mt = ((inst.part[mu] + 1 + rng.integers(0, inst.k - 1, t)) % inst.k).astype(np.int32)
    return mu, mt


@pytest.mark.parametrize("name,make", INSTANCES, ids=[c[0] for c in INSTANCES])
def test_move_gains_and_best_prefix(H, name, make):
    import torch
    inst = make()
    h = _oracle_hg(inst)
    k = inst.k
    g = H.hg_load_csr(inst.n, inst.eptr, inst.pins, inst.c, inst.w, k_max=k)
    st = H.State(g, k, inst.part)
    H.hg_compute_pincounts(g, st)
    ws = H.moves_workspace(g, k)
    rng = np.random.default_rng(7)
    total = int(inst.c.astype(np.int64).sum())
    for t in (1, 37, inst.n // 3, inst.n):
        mu, mt = _sequence(rng, inst, t)
        got = H.hg_move_gains(g, k, st.part, st.phi, mu, mt, ws)
        want = O.move_gains(h, k, inst.part, mu, mt)
        assert np.array_equal(got.cpu().numpy(), want), (name, t)
        # the partition state is read, not changed
        assert np.array_equal(st.part.cpu().numpy(), inst.part)
        for lm in (total // k + total // (10 * k), total):
            blen, bgain = H.hg_best_prefix(g, k, lm, st.part, st.block_w, mu, mt, got, ws)
            assert (int(blen.item()), int(bgain.item())) == O.best_prefix(
                h, k, lm, inst.part, mu, mt, want), (name, t, lm)
    H.hg_sync_status(g)
    # a vertex twice raises the device flag
    mu, mt = _sequence(rng, inst, 5)
    mu[3] = mu[1]
    H.hg_move_gains(g, k, st.part, st.phi, mu, mt, ws)
    with pytest.raises(H.HgError) as ei:
        H.hg_sync_status(g)
    assert ei.value.code == H.HG_ERR_INVALID
    torch.cuda.synchronize()


@pytest.mark.parametrize("name,make", INSTANCES, ids=[c[0] for c in INSTANCES])
def test_monotone_rounds_bit_exact(H, name, make):
    import torch
    inst = make()
    h = _oracle_hg(inst)
    k = inst.k
    g = H.hg_load_csr(inst.n, inst.eptr, inst.pins, inst.c, inst.w, k_max=k)
    L = H.hg_max_block_weight(g, k, inst.eps)
    st = H.State(g, k, inst.part)
    H.hg_compute_pincounts(g, st)
    ws = H.moves_workspace(g, k)
    part_o = inst.part.copy()
    elig_o = np.ones(inst.n, np.uint8)
    stats = torch.zeros(H.STATS_WORDS, dtype=torch.int64, device="cuda")
    cut = 0
    for r in range(inst.rounds):
        km_before = int(st.km1.item())
        H.hg_lp_round_exact(g, st, L, stats, ws)
        torch.cuda.synchronize()
        part_o, elig_o, moved_o, st_o, napp = O.lp_round_exact(h, k, L, part_o, elig_o)
        sg = H.stats_to_dicts(stats)[0]
        assert sg["km1_delta_recomputed"] == sg["km1_delta"], (r, sg)
        sg.pop("km1_delta_recomputed")
        assert sg == st_o, (name, r, sg, st_o)
        assert sg["km1_delta"] >= 0 and sg["km1_after"] == km_before - sg["km1_delta"]
        assert np.array_equal(st.part.cpu().numpy(), part_o), r
        assert np.array_equal(st.moved.cpu().numpy(), moved_o), r
        assert np.array_equal(st.eligible.cpu().numpy(), elig_o), r
        _check_state(H, g, st, h, k, part_o)
        cut += sg["approved"] < napp
    H.hg_sync_status(g)


def test_refine_exact_matches_oracle(H):
    import torch
    inst = synth.random_power_law(42, 20000, 19000, 16, hi=32, unit=False, rounds=6)
    h = _oracle_hg(inst)
    g = H.hg_load_csr(inst.n, inst.eptr, inst.pins, inst.c, inst.w, k_max=16)
    L = H.hg_max_block_weight(g, 16, inst.eps)
    part_o, stats_o, km_o = O.refine_exact(h, 16, L, inst.rounds, inst.part)
    st = H.State(g, 16, inst.part)
    ws = H.moves_workspace(g, 16)
    stats = torch.zeros(inst.rounds * H.STATS_WORDS, dtype=torch.int64, device="cuda")
    for rep in range(2):
        st.part.copy_(torch.as_tensor(inst.part))
        H.hg_refine_exact(g, st, inst.eps, inst.rounds, stats, ws)
        torch.cuda.synchronize()
        assert np.array_equal(st.part.cpu().numpy(), part_o)
        got = H.stats_to_dicts(stats)
        prev = None
        for r in range(inst.rounds):
            got[r].pop("km1_delta_recomputed")
            assert got[r] == stats_o[r], (rep, r)
            assert prev is None or got[r]["km1_after"] <= prev
            prev = got[r]["km1_after"]
        assert int(st.km1.item()) == km_o
    H.hg_sync_status(g)
