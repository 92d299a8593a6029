"""GPU parity of batched refinement (hg_batch_* through the C ABI).

A batch must give every member exactly what hg_refine gives it alone, and
what the oracle computes, whatever the schedule, the placement on XCDs and
the other members.  Members mix sizes (so that some are spread over all XCDs
and some sit on one), k from 2 to 256, unit and weighted nets and vertices
with the wavefront (heavy) path.
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


def _mixed(seed=11, count=14):
    insts = synth.batch_instances(seed=seed, count=count, n_lo=300, n_hi=12000,
                                  ks=(2, 3, 8, 17, 32, 64, 100, 128, 256), rounds=4)
    insts.append(synth.random_power_law(77, 60000, 57000, 16, hi=24, unit=False, rounds=4))
    insts.append(_hub_instance(8, 6000, 5000, 16, 400, True))
    insts.append(_hub_instance(9, 5000, 4000, 70, 500, True))
    insts.append(synth.random_power_law(78, 3000, 2800, 5, hi=12, unit=False, rounds=4))
    return insts


def _members(H, insts, rounds):
    import torch
    out = []
    for inst in insts:
        g = H.hg_load_csr(inst.n, inst.eptr, inst.pins, inst.c, inst.w, k_max=inst.k)
        st = H.State(g, inst.k, inst.part)
        stats = torch.zeros(max(rounds, 1) * H.STATS_WORDS, dtype=torch.int64, device="cuda")
        out.append(H.Member(g, st, inst.eps, stats))
    return out


def _snapshot(mb):
    st = mb.st
    return [st.part.cpu().numpy(), st.phi.cpu().numpy(), st.netstate.cpu().numpy(),
            st.block_w.cpu().numpy(), st.km1.cpu().numpy(), st.eligible.cpu().numpy(),
            mb.stats.cpu().numpy()]


@pytest.fixture(scope="module")
def mixed():
    return _mixed()


@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_refine_matches_oracle(H, mixed, use_graph):
    import torch
    R = 4
    mem = _members(H, mixed, R)
    b = H.hg_batch_create(mem)
    for rep in range(2 if use_graph else 1):      # graph replays agree too
        for inst, mb in zip(mixed, mem):
            mb.st.part.copy_(torch.as_tensor(inst.part))
            mb.stats.zero_()
        H.hg_batch_refine(b, R, use_graph=use_graph)
        torch.cuda.synchronize()
        for inst, mb in zip(mixed, mem):
            h = _oracle_hg(inst)
            L = O.lmax(O.total_vertex_weight(h), inst.k, inst.eps)
            part_o, stats_o, km_o = O.refine(h, inst.k, L, R, inst.part)
            assert np.array_equal(mb.st.part.cpu().numpy(), part_o), (inst.name, rep)
            got = H.stats_to_dicts(mb.stats)
            for r in range(R):
                assert got[r]["km1_delta_recomputed"] == got[r]["km1_delta"]
                got[r].pop("km1_delta_recomputed")
                assert got[r] == stats_o[r], (inst.name, rep, r)
            assert int(mb.st.km1.item()) == km_o
            _check_state(H, mb.g, mb.st, h, inst.k, part_o)
    b.free()
    for mb in mem:
        H.hg_sync_status(mb.g)


def test_batch_rounds_match_oracle_round_by_round(H, mixed):
    import torch
    R = 3
    mem = _members(H, mixed, R)
    b = H.hg_batch_create(mem)
    H.hg_batch_start(b)
    parts = [inst.part.copy() for inst in mixed]
    eligs = [np.ones(inst.n, np.uint8) for inst in mixed]
    hs = [_oracle_hg(inst) for inst in mixed]
    for r in range(R):
        H.hg_batch_round(b, r)
        torch.cuda.synchronize()
        for i, (inst, mb) in enumerate(zip(mixed, mem)):
            L = O.lmax(O.total_vertex_weight(hs[i]), inst.k, inst.eps)
            parts[i], eligs[i], _, st_o = O.lp_round(hs[i], inst.k, L, parts[i], eligs[i])
            sg = H.stats_to_dicts(mb.stats)[r]
            sg.pop("km1_delta_recomputed")
            assert sg == st_o, (inst.name, r)
            assert np.array_equal(mb.st.part.cpu().numpy(), parts[i]), (inst.name, r)
            assert np.array_equal(mb.st.eligible.cpu().numpy(), eligs[i]), (inst.name, r)
    b.free()


def test_batch_equals_sequential_and_schedules_agree(H):
    """Bit-identical state to one-at-a-time hg_refine, under the default, an
    odd hand-picked and the autotuned schedule."""
    import torch
    R = 5
    insts = synth.batch_instances(seed=21, count=40, n_lo=1000, n_hi=150000, rounds=R)
    seq = _members(H, insts, R)
    for mb in seq:
        H.hg_refine(mb.g, mb.st, mb.eps, R, mb.stats, use_graph=True)
    torch.cuda.synchronize()
    want = [_snapshot(mb) for mb in seq]
    del seq
    odd = [dict(select_chunks=3, finalize_chunks=5, count_chunks=7, net_lanes=32)] * 4
    for sched in (None, odd, "tuned"):
        mem = _members(H, insts, R)
        b = H.hg_batch_create(mem, sched=None if sched == "tuned" else sched)
        if sched == "tuned":
            before = [mb.st.part.cpu().numpy() for mb in mem]
            tuned = H.hg_batch_autotune(b, repeats=1)
            assert len(tuned) == H.HG_SIZE_CLASSES
            assert H.hg_batch_get_schedule(b) == tuned
            for mb, p0 in zip(mem, before):              # partitions restored
                assert np.array_equal(mb.st.part.cpu().numpy(), p0)
        H.hg_batch_refine(b, R, use_graph=True)
        torch.cuda.synchronize()
        for inst, mb, w in zip(insts, mem, want):
            got = _snapshot(mb)
            for a, c in zip(got, w):
                assert np.array_equal(a, c), (inst.name, sched)
        b.free()


def test_batch_invalid_members(H):
    import torch
    insts = synth.batch_instances(seed=5, count=2, n_lo=500, n_hi=900, rounds=1)
    mem = _members(H, insts, 1)
    with pytest.raises(H.HgError) as ei:                      # one graph twice
        H.hg_batch_create([mem[0], H.Member(mem[0].g, mem[1].st, 0.03, mem[1].stats)])
    assert ei.value.code == H.HG_ERR_INVALID
    with pytest.raises(H.HgError) as ei:                      # eps out of range
        H.hg_batch_create([H.Member(mem[0].g, mem[0].st, 1.5, mem[0].stats)])
    assert ei.value.code == H.HG_ERR_INVALID
    with pytest.raises(H.HgError) as ei:                      # table too small
        H.hg_batch_create(mem, table=torch.empty(16, dtype=torch.uint8, device="cuda"))
    assert ei.value.code == H.HG_ERR_WORKSPACE
    bad = [dict(select_chunks=0, finalize_chunks=1, count_chunks=1, net_lanes=0)] * 4
    with pytest.raises(H.HgError) as ei:                      # schedule out of range
        H.hg_batch_create(mem, sched=bad)
    assert ei.value.code == H.HG_ERR_INVALID
