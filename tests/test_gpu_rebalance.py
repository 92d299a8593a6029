"""GPU parity of the rebalancer (hg_rebalance), through the C ABI, against
the oracle's rebalancing rounds: partition, moved flags, eligible flags,
round records and the pin-count state, all exactly equal, round by round.
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


def _overload(inst, seed, frac, blocks=(0,)):
    """The instance with a random `frac` of the vertices piled into `blocks`."""
    rng = np.random.default_rng(seed)
    part = inst.part.copy()
    pick = rng.random(inst.n) < frac
    part[pick] = rng.choice(np.array(blocks, np.int32), int(pick.sum()))
    return part


def _instances():
    yield "plaw-k2-u", lambda: synth.random_power_law(401, 9000, 8500, 2, hi=24), (0,), 0.3
    yield "plaw-k7-w", lambda: synth.random_power_law(402, 7000, 6600, 7, hi=16, unit=False), \
        (0, 3), 0.25
    yield "plaw-k64-u", lambda: synth.random_power_law(403, 8000, 7800, 64, hi=24), \
        (5,), 0.1
    yield "plaw-k200-w", lambda: synth.random_power_law(404, 6000, 5600, 200, hi=12,
                                                        unit=False), (0, 1, 2), 0.05
    yield "plaw-k256-u", lambda: synth.random_power_law(405, 5000, 5200, 256, hi=10), \
        (255,), 0.05
    yield "band-k16", lambda: synth.sparse_matrix(16, seed=406, rows=30000, cols=30000,
                                                  band=1000), (2,), 0.2
    yield "hub-k16-w", lambda: _hub_instance(8, 6000, 5000, 16, 400, True), (0, 15), 0.2
    yield "hub-k3-u", lambda: _hub_instance(9, 5000, 4000, 3, 600, False), (1,), 0.4


INSTANCES = list(_instances())
IDS = [c[0] for c in INSTANCES]


@pytest.mark.parametrize("name,make,blocks,frac", INSTANCES, ids=IDS)
def test_rebalance_rounds_bit_exact(H, name, make, blocks, frac):
    import torch
    inst = make()
    h = _oracle_hg(inst)
    k = inst.k
    part0 = _overload(inst, 7, frac, blocks)
    g = H.hg_load_csr(inst.n, inst.eptr, inst.pins, inst.c, inst.w, k_max=k)
    L = H.hg_max_block_weight(g, k, inst.eps)
    st = H.State(g, k, part0)
    rng = np.random.default_rng(8)
    elig0 = (rng.random(inst.n) < 0.3).astype(np.uint8)
    st.eligible.copy_(torch.as_tensor(elig0))
    H.hg_compute_pincounts(g, st)
    ws = H.rebalance_workspace(g, k)
    ws.fill_(0xA5)                        # nothing may read what a round does not write
    stats = torch.zeros(H.STATS_WORDS, dtype=torch.int64, device="cuda")
    part_o, elig_o = part0.copy(), elig0.copy()
    moves = 0
    for r in range(4):
        H.hg_rebalance(g, st, L, 1, stats, ws)
        torch.cuda.synchronize()
        part_o, elig_o, moved_o, st_o = O.rebalance_round(h, k, L, part_o, elig_o)
        sg = H.stats_to_dicts(stats)[0]
        assert sg.pop("km1_delta_recomputed") == sg["km1_delta"], (name, r)
        assert sg == st_o, (name, r, sg, st_o)
        assert np.array_equal(st.part.cpu().numpy(), part_o), (name, r)
        assert np.array_equal(st.moved.cpu().numpy(), moved_o), (name, r)
        assert np.array_equal(st.eligible.cpu().numpy(), elig_o), (name, r)
        _check_state(H, g, st, h, k, part_o)
        moves += sg["approved"]
    H.hg_sync_status(g)
    assert moves > 0, name


@pytest.mark.parametrize("name,make,blocks,frac", INSTANCES[1:2] + INSTANCES[6:7],
                         ids=IDS[1:2] + IDS[6:7])
def test_rebalance_driver_matches_oracle(H, name, make, blocks, frac):
    import torch
    inst = make()
    h = _oracle_hg(inst)
    k = inst.k
    part0 = _overload(inst, 9, frac, blocks)
    g = H.hg_load_csr(inst.n, inst.eptr, inst.pins, inst.c, inst.w, k_max=k)
    L = H.hg_max_block_weight(g, k, inst.eps)
    part_o, elig_o, stats_o, km_o = O.rebalance(h, k, L, 5, part0, np.ones(inst.n, np.uint8))
    st = H.State(g, k, part0)
    ws = H.rebalance_workspace(g, k)
    stats = torch.zeros(5 * H.STATS_WORDS, dtype=torch.int64, device="cuda")
    for rep in range(2):
        st.part.copy_(torch.as_tensor(part0))
        st.eligible.fill_(1)
        H.hg_compute_pincounts(g, st)
        H.hg_rebalance(g, st, L, 5, stats, ws)
        torch.cuda.synchronize()
        assert np.array_equal(st.part.cpu().numpy(), part_o), (name, rep)
        got = H.stats_to_dicts(stats)
        for r in range(5):
            got[r].pop("km1_delta_recomputed")
            assert got[r] == stats_o[r], (name, rep, r)
        assert int(st.km1.item()) == km_o
    H.hg_sync_status(g)


def test_balanced_partition_is_left_alone(H):
    import torch
    inst = synth.random_power_law(407, 6000, 5500, 8, hi=16, unit=False)
    g = H.hg_load_csr(inst.n, inst.eptr, inst.pins, inst.c, inst.w, k_max=8)
    L = H.hg_max_block_weight(g, 8, inst.eps)
    st = H.State(g, 8, inst.part)
    H.hg_compute_pincounts(g, st)
    assert int(st.block_w.max().item()) <= L
    ws = H.rebalance_workspace(g, 8)
    stats = torch.zeros(2 * H.STATS_WORDS, dtype=torch.int64, device="cuda")
    km = int(st.km1.item())
    H.hg_rebalance(g, st, L, 2, stats, ws)
    torch.cuda.synchronize()
    assert np.array_equal(st.part.cpu().numpy(), inst.part)
    for s in H.stats_to_dicts(stats):
        assert s["eligible"] == s["approved"] == s["candidates"] == 0
        assert s["km1_after"] == km
    with pytest.raises(H.HgError) as ei:          # workspace too small
        H.hg_rebalance(g, st, L, 1, stats, ws[:1024])
    assert ei.value.code == H.HG_ERR_WORKSPACE
    H.hg_sync_status(g)
