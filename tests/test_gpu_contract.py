"""GPU parity of the contraction (hg_contract), through the C ABI, against
the oracle: map, coarse weights and the coarse net CSR exactly equal, on
several clusterings, including the full sparse-matrix workload; the coarse
hypergraph loads and keeps km1 of projected partitions.
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


def _with_duplicates(inst, seed):
    """The instance with a seeded 20% of its nets repeated (identical nets)."""
    rng = np.random.default_rng(seed)
    nets = [inst.pins[inst.eptr[e]:inst.eptr[e + 1]] for e in range(inst.m)]
    extra = rng.choice(inst.m, size=inst.m // 5)
    nets = nets + [nets[e] for e in extra]
    order = rng.permutation(len(nets))
    nets = [nets[e] for e in order]
    w = None
    if inst.w is not None:
        w = np.concatenate([inst.w, inst.w[extra]])[order].astype(np.int32)
    eptr = np.zeros(len(nets) + 1, np.int64)
    eptr[1:] = np.cumsum([len(x) for x in nets])
    return synth.Instance(inst.name + "-dup", inst.n, eptr, np.concatenate(nets).astype(np.int32),
                          inst.c, w, inst.part, inst.k, inst.eps, inst.rounds)


def _with_huge_nets(seed):
    """A power-law hypergraph plus nets of 100, 5,000, 9,000 and 20,000 pins
    (longer than one thread's sort, and than the LDS sort), one of them twice."""
    rng = np.random.default_rng(seed)
    base = synth.random_power_law(seed, 30000, 20000, 4, hi=32, unit=False)
    nets = [base.pins[base.eptr[e]:base.eptr[e + 1]] for e in range(base.m)]
    for size in (100, 5000, 9000, 20000, 9000):
        nets.append(np.sort(rng.choice(base.n, size=size, replace=False)).astype(np.int32))
    nets.append(nets[-2].copy())
    w = np.concatenate([base.w, rng.integers(1, 50, 6)]).astype(np.int32)
    eptr = np.zeros(len(nets) + 1, np.int64)
    eptr[1:] = np.cumsum([len(x) for x in nets])
    return synth.Instance("huge", base.n, eptr, np.concatenate(nets).astype(np.int32), base.c, w,
                          base.part, 4, 0.03, 3)


def _clusterings(inst):
    rng = np.random.default_rng(5)
    n = inst.n
    yield "neighbour", synth.neighbour_clusters(inst, 3)
    yield "neighbour-all", synth.neighbour_clusters(inst, 4, join=1.0)
    yield "few", rng.integers(0, max(2, n // 500), n).astype(np.int32)
    yield "identity", np.arange(n, dtype=np.int32)
    yield "one", np.full(n, n - 1, np.int32)
    yield "anywhere", rng.choice(n, size=n).astype(np.int32)


def _instances():
    yield "plaw-u", lambda: synth.random_power_law(501, 9000, 8500, 2, hi=24)
    yield "plaw-w-dup", lambda: _with_duplicates(
        synth.random_power_law(502, 7000, 6600, 7, hi=16, unit=False), 1)
    yield "band", lambda: synth.sparse_matrix(16, seed=503, rows=30000, cols=30000, band=1000)
    yield "hub-w", lambda: _hub_instance(8, 6000, 5000, 16, 400, True)
    yield "huge-nets", lambda: _with_huge_nets(506)


INSTANCES = list(_instances())


def _check(H, g, inst, cl, what):
    import torch
    h = _oracle_hg(inst)
    mp_o, hc = O.contract(h, cl)
    out = H.Coarse(g)
    ws = H.contract_workspace(g)
    ws.fill_(0x5A)                         # nothing may read what the call does not write
    H.hg_contract(g, cl, out, ws)
    torch.cuda.synchronize()
    H.hg_sync_status(g)
    assert out.read_sizes() == (hc.n, hc.m, hc.P), what
    mp, cv, ce, cpn, cw = (x.cpu().numpy() for x in out.views())
    assert np.array_equal(mp, mp_o), what
    assert np.array_equal(cv, hc.c), what
    assert np.array_equal(ce, hc.eptr), what
    assert np.array_equal(cpn, hc.pins), what
    assert np.array_equal(cw, hc.w), what
    return out, hc, mp_o


@pytest.mark.parametrize("name,make", INSTANCES, ids=[c[0] for c in INSTANCES])
def test_contract_matches_oracle(H, name, make):
    inst = make()
    g = H.hg_load_csr(inst.n, inst.eptr, inst.pins, inst.c, inst.w, k_max=2)
    for cname, cl in _clusterings(inst):
        _check(H, g, inst, cl, (name, cname))
        _check(H, g, inst, cl, (name, cname, "again"))   # a second call on used buffers


def test_coarse_graph_keeps_km1(H):
    import torch
    inst = synth.random_power_law(504, 20000, 19000, 8, hi=32, unit=False)
    g = H.hg_load_csr(inst.n, inst.eptr, inst.pins, inst.c, inst.w, k_max=8)
    out, hc, mp = _check(H, g, inst, synth.neighbour_clusters(inst, 7), "km1")
    _, cv, ce, cpn, cw = out.views()
    gc = H.hg_load_csr(hc.n, ce, cpn, cv, cw, k_max=8)
    rng = np.random.default_rng(3)
    for _ in range(3):
        cp = rng.integers(0, 8, hc.n).astype(np.int32)
        sc = H.State(gc, 8, cp)
        H.hg_compute_pincounts(gc, sc)
        sf = H.State(g, 8, cp[mp])
        H.hg_compute_pincounts(g, sf)
        torch.cuda.synchronize()
        assert int(sc.km1.item()) == int(sf.km1.item())
        assert torch.equal(sc.block_w, sf.block_w)


def test_full_sparse_matrix_workload(H):
    inst = synth.sparse_matrix(8)
    g = H.hg_load_csr(inst.n, inst.eptr, inst.pins, inst.c, inst.w, k_max=8)
    _check(H, g, inst, synth.neighbour_clusters(inst), "sparse-matrix")


def test_contract_errors(H):
    import torch
    inst = synth.random_power_law(505, 500, 400, 4, hi=8)
    g = H.hg_load_csr(inst.n, inst.eptr, inst.pins, inst.c, inst.w, k_max=4)
    out = H.Coarse(g)
    ws = H.contract_workspace(g)
    bad = np.arange(inst.n, dtype=np.int32)
    bad[7] = inst.n
    H.hg_contract(g, bad, out, ws)
    with pytest.raises(H.HgError) as ei:
        H.hg_sync_status(g)
    assert "cluster id" in str(ei.value)
    heavy = H.hg_load_csr(inst.n, inst.eptr, inst.pins, np.full(inst.n, 2**30, np.int32),
                          inst.w, k_max=4)
    H.hg_contract(heavy, np.zeros(inst.n, np.int32), H.Coarse(heavy), ws)
    with pytest.raises(H.HgError) as ei:
        H.hg_sync_status(heavy)
    assert "2^31" in str(ei.value)
    with pytest.raises(H.HgError) as ei:
        H.hg_contract(g, np.arange(inst.n), out, ws[:256])
    assert ei.value.code == H.HG_ERR_WORKSPACE
    torch.cuda.synchronize()
