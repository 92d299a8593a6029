"""hg_lp_round_noalloc (round scratch in the library's fixed device array)
against hg_lp_round (round scratch in the graph's workspace): the same
kernels, so every output must be bit-identical.  Two graphs in a row, the
second smaller, so the second call runs on what the first left in the array;
plus the size limit, which is rejected on the host before anything is
enqueued."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2010_10272_amd import hgref
    return hgref


def _state_arrays(st, stats):
    return [st.part, st.phi, st.netstate, st.block_w, st.km1, st.eligible, st.moved, stats]


def _rounds_agree(H, inst, rounds):
    import torch
    k = inst.k
    g = H.hg_load_csr(inst.n, inst.eptr, inst.pins, inst.c, inst.w, k_max=k)
    L = H.hg_max_block_weight(g, k, inst.eps)
    a = H.State(g, k, inst.part)
    b = H.State(g, k, inst.part)
    H.hg_compute_pincounts(g, a)
    H.hg_compute_pincounts(g, b)
    sa = torch.zeros(H.STATS_WORDS, dtype=torch.int64, device="cuda")
    sb = torch.zeros(H.STATS_WORDS, dtype=torch.int64, device="cuda")
    moves = 0
    for r in range(rounds):
        H.hg_lp_round(g, a, L, sa)
        H.hg_lp_round_noalloc(g, b, L, sb)
        torch.cuda.synchronize()
        for x, y in zip(_state_arrays(a, sa), _state_arrays(b, sb)):
            assert torch.equal(x, y), (inst.name, r)
        moves += H.stats_to_dicts(sa)[0]["approved"]
    H.hg_sync_status(g)
    g.free()
    return moves


def test_noalloc_round_equals_workspace_round_twice_shrinking(H):
    big = synth.random_power_law(71, 300_000, 280_000, 32, hi=40, unit=False, rounds=3)
    small = synth.random_power_law(72, 20_000, 19_000, 8, hi=24, unit=True, rounds=3)
    assert _rounds_agree(H, big, 3) > 0
    assert _rounds_agree(H, small, 3) > 0


def test_noalloc_heavy_vertices_and_wide_k(H):
    inst = synth.random_power_law(73, 9_000, 8_000, 200, hi=24, unit=False, rounds=2)
    assert _rounds_agree(H, inst, 2) >= 0


def test_noalloc_rejects_graphs_beyond_the_limit(H):
    import torch
    n = (1 << 20) + 5
    m = 1000
    rng = np.random.default_rng(3)
    pins = np.concatenate([rng.choice(n, 4, replace=False) for _ in range(m)]).astype(np.int32)
    eptr = np.arange(0, 4 * m + 1, 4, dtype=np.int64)
    g = H.hg_load_csr(n, eptr, pins, k_max=4)
    st = H.State(g, 4, np.zeros(n, np.int32))
    H.hg_compute_pincounts(g, st)
    stats = torch.zeros(H.STATS_WORDS, dtype=torch.int64, device="cuda")
    part0 = st.part.clone()
    with pytest.raises(H.HgError) as ei:
        H.hg_lp_round_noalloc(g, st, H.hg_max_block_weight(g, 4, 0.03), stats)
    assert ei.value.code == H.HG_ERR_UNSUPPORTED
    torch.cuda.synchronize()
    assert torch.equal(st.part, part0)
    g.free()
