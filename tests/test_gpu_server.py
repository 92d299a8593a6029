"""GPU tests of the request server (hg_server_* through the C ABI).

Each job's result must be what hg_refine gives the same job alone (and what
the oracle gives), whatever else shares the steps with it: other jobs of
every size class and k, jobs admitted later because memory ran out, jobs
that fail their load checks.
"""
import numpy as np
import pytest

import synth
from oracle import oracle as O

from .test_gpu_parity import _hub_instance, _oracle_hg

pytestmark = pytest.mark.gpu

DRAIN_MS = 120000.0


@pytest.fixture(scope="module")
def H():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2010_10272_amd import hgref
    return hgref


def _jobs():
    insts = synth.batch_instances(seed=31, count=10, n_lo=400, n_hi=40000,
                                  ks=(2, 4, 8, 32, 128, 256), rounds=6)
    insts.append(_hub_instance(8, 6000, 5000, 16, 400, True))
    insts.append(synth.random_power_law(79, 20000, 19000, 9, hi=20, unit=False, rounds=3))
    insts.append(synth.vlsi_grid(seed=3, side=300, height=200, m=63000, k=16, rounds=5))
    return insts


@pytest.fixture(scope="module")
def jobs():
    return _jobs()


@pytest.fixture(scope="module")
def alone(H, jobs):
    """Each job refined alone with hg_refine: (part, stats dicts, km1)."""
    import torch
    out = []
    for inst in jobs:
        g = H.hg_load_csr(inst.n, inst.eptr, inst.pins, inst.c, inst.w, k_max=inst.k)
        st = H.State(g, inst.k, inst.part)
        stats = torch.zeros(inst.rounds * H.STATS_WORDS, dtype=torch.int64, device="cuda")
        H.hg_refine(g, st, inst.eps, inst.rounds, stats, use_graph=False)
        torch.cuda.synchronize()
        out.append((st.part.cpu().numpy(), H.stats_to_dicts(stats), int(st.km1.item())))
        g.free()
    return out


def _submit_all(H, srv, insts, order):
    ids = {}
    for i in order:
        x = insts[i]
        ids[i] = H.hg_server_submit(srv, x.n, x.eptr, x.pins, x.part, x.k, x.rounds, x.eps,
                                    vwgt=x.c, ewgt=x.w)
    return ids


def _check_results(H, srv, insts, ids, alone):
    for i, jid in ids.items():
        info = H.hg_server_info(srv, jid)
        assert info["state"] == H.HG_REQ_DONE and info["status"] == H.HG_OK, (insts[i].name, info)
        assert info["arrival_ms"] <= info["admit_ms"] <= info["loaded_ms"] <= info["done_ms"]
        part, stats, km1 = H.hg_server_result(srv, jid)
        want_part, want_stats, want_km1 = alone[i]
        assert np.array_equal(part.numpy(), want_part), insts[i].name
        assert stats == want_stats, insts[i].name
        assert km1 == want_km1, insts[i].name


def test_alone_results_match_oracle(H, jobs, alone):
    """Pin the reference itself: hg_refine alone equals the oracle."""
    for inst, (part, stats, km1) in zip(jobs, alone):
        h = _oracle_hg(inst)
        L = O.lmax(O.total_vertex_weight(h), inst.k, inst.eps)
        part_o, stats_o, km_o = O.refine(h, inst.k, L, inst.rounds, inst.part)
        assert np.array_equal(part, part_o), inst.name
        assert km1 == km_o
        for r in range(inst.rounds):
            s = dict(stats[r])
            s.pop("km1_delta_recomputed")
            assert s == stats_o[r], (inst.name, r)


@pytest.mark.parametrize("order,big_pins", [("given", 0), ("reversed", 0), ("interleaved", 0),
                                             ("given", 100000), ("interleaved", 100000)])
def test_server_mix_equals_alone(H, jobs, alone, order, big_pins):
    n = len(jobs)
    idx = {"given": list(range(n)), "reversed": list(range(n))[::-1],
           "interleaved": list(range(0, n, 2)) + list(range(1, n, 2))}[order]
    if big_pins:                                    # both lanes get jobs
        assert any(x.P >= big_pins for x in jobs) and any(x.P < big_pins for x in jobs)
    srv = H.hg_server_create(1 << 30, table_bytes=8 << 20, max_active=64, big_pins=big_pins)
    ids = _submit_all(H, srv, jobs, idx)
    assert H.hg_server_drain(srv, DRAIN_MS) == 0
    _check_results(H, srv, jobs, ids, alone)
    st = H.hg_server_get_stats(srv)
    assert st["completed"] == n and st["failed"] == 0
    assert st["member_rounds"] == sum(x.rounds for x in jobs)
    assert st["max_members"] > 1            # jobs really shared steps
    srv.free()


def test_server_tiny_budget_one_at_a_time(H, jobs, alone):
    """Job memory that fits only the largest job: admission binds, every job
    still finishes with the same result."""
    need = max(H.hg_request_bytes(x.n, x.m, x.P, x.k, x.rounds, True, True) for x in jobs)
    srv = H.hg_server_create((4 << 20) + need, table_bytes=4 << 20, max_active=64)
    ids = _submit_all(H, srv, jobs, list(range(len(jobs))))
    assert H.hg_server_drain(srv, DRAIN_MS) == 0
    _check_results(H, srv, jobs, ids, alone)
    st = H.hg_server_get_stats(srv)
    assert st["peak_bytes"] <= need
    srv.free()


def test_server_max_active_and_failures(H, jobs, alone):
    import torch
    srv = H.hg_server_create(1 << 30, table_bytes=8 << 20, max_active=2)
    good = _submit_all(H, srv, jobs, [0, 1, 2])
    bad_pins = H.hg_server_submit(srv, 3, np.array([0, 2, 4]), np.array([0, 1, 1, 7]),
                                  np.zeros(3, np.int32), 2, 2, 0.03)    # pin out of range
    big = synth.random_power_law(3, 300000, 300000, 64, rounds=2)
    too_big = None
    srv2 = H.hg_server_create(64 << 20, table_bytes=4 << 20, max_active=4)
    too_big = H.hg_server_submit(srv2, big.n, big.eptr, big.pins, big.part, big.k, 2, 0.03)
    more = _submit_all(H, srv, jobs, [3, 4])
    assert H.hg_server_drain(srv, DRAIN_MS) == 0
    assert H.hg_server_drain(srv2, DRAIN_MS) == 0
    good.update(more)
    _check_results(H, srv, jobs, good, alone)
    info = H.hg_server_info(srv, bad_pins)
    assert info["state"] == H.HG_REQ_DONE and info["status"] == H.HG_ERR_INVALID
    info = H.hg_server_info(srv2, too_big)
    assert info["state"] == H.HG_REQ_DONE and info["status"] == H.HG_ERR_WORKSPACE
    st = H.hg_server_get_stats(srv)
    assert st["max_members"] <= 2 and st["failed"] == 1 and st["completed"] == 5
    with pytest.raises(H.HgError):                       # argument checks on the host
        H.hg_server_submit(srv, 3, np.array([0, 2, 4]), np.array([0, 1, 1, 2]),
                           np.zeros(3, np.int32), 1, 2, 0.03)
    srv.free()
    srv2.free()
    torch.cuda.synchronize()
