"""Python view of the CPU oracle (``hgoracle.c``), numpy in, numpy out.

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` use this module.  The product path (the HIP
library and its binding) never imports it.

Every function here is a thin ctypes call into the single-threaded C oracle;
see ``hgoracle.c`` for the definitions each one writes out.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hgoracle.c")
_LIB_PATH = os.path.join(_HERE, "libhgoracle.so")
_lib = None

OR_OK = 0
OR_ERR_INVALID = -1

STATS_FIELDS = ("eligible", "boundary", "candidates", "approved", "moved_pins",
                "touched_nets", "km1_delta", "km1_after", "max_block_weight", "active_pins",
                "touched_pins")


class RoundStats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in STATS_FIELDS]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f in STATS_FIELDS}


CC = "gcc"
CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-Wall"]


def build(force=False):
    """Compile the oracle with gcc into oracle/libhgoracle.so."""
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call([CC] + CFLAGS + ["-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        build()
        _lib = ctypes.CDLL(_LIB_PATH)
        i32, i64, vp, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_double
        _lib.or_check_hypergraph.argtypes = [i32, i32, i64, vp, vp, vp, vp]
        _lib.or_check_hypergraph.restype = ctypes.c_int
        _lib.or_check_partition.argtypes = [i32, vp, i32]
        _lib.or_incidence.argtypes = [i32, i32, vp, vp, vp, vp]
        _lib.or_pin_counts.argtypes = [i32, vp, vp, vp, i32, vp]
        _lib.or_connectivity.argtypes = [i32, i32, vp, vp, vp]
        _lib.or_block_weights.argtypes = [i32, vp, vp, i32, vp]
        _lib.or_km1.argtypes = [i32, vp, vp]
        _lib.or_km1.restype = i64
        _lib.or_lmax.argtypes = [i64, i32, dbl]
        _lib.or_lmax.restype = i64
        _lib.or_gains.argtypes = [i32, vp, vp, vp, vp, i32, vp, vp, vp]
        _lib.or_gain_cache.argtypes = [i32, vp, vp, vp, vp, i32, vp, vp, vp, vp]
        _lib.or_lp_round.argtypes = [i32, i32, vp, vp, vp, vp, vp, vp, i32, i64, vp, vp,
                                     vp, ctypes.POINTER(RoundStats)]
        _lib.or_lp_round.restype = ctypes.c_int
        _lib.or_refine.argtypes = [i32, i32, vp, vp, vp, vp, i32, i64, i32, vp,
                                   ctypes.POINTER(RoundStats), ctypes.POINTER(i64)]
        _lib.or_refine.restype = ctypes.c_int
        _lib.or_move_gains.argtypes = [i32, i32, vp, vp, vp, vp, vp, i32, vp, i32, vp, vp, vp]
        _lib.or_move_gains.restype = ctypes.c_int
        _lib.or_best_prefix.argtypes = [i32, vp, i32, i64, vp, i32, vp, vp, vp,
                                        ctypes.POINTER(i32), ctypes.POINTER(i64)]
        _lib.or_best_prefix.restype = None
        _lib.or_lp_round_exact.argtypes = [i32, i32, vp, vp, vp, vp, vp, vp, i32, i64, vp, vp,
                                           vp, ctypes.POINTER(RoundStats), ctypes.POINTER(i64)]
        _lib.or_lp_round_exact.restype = ctypes.c_int
        _lib.or_rebalance_round.argtypes = [i32, i32, vp, vp, vp, vp, vp, vp, i32, i64, vp,
                                            vp, vp, ctypes.POINTER(RoundStats)]
        _lib.or_rebalance_round.restype = ctypes.c_int
        _lib.or_rebalance.argtypes = [i32, i32, vp, vp, vp, vp, i32, i64, i32, vp, vp,
                                      ctypes.POINTER(RoundStats), ctypes.POINTER(i64)]
        _lib.or_rebalance.restype = ctypes.c_int
        _lib.or_contract.argtypes = [i32, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        _lib.or_contract.restype = ctypes.c_int
        _lib.or_refine_exact.argtypes = [i32, i32, vp, vp, vp, vp, i32, i64, i32, vp,
                                         ctypes.POINTER(RoundStats), ctypes.POINTER(i64)]
        _lib.or_refine_exact.restype = ctypes.c_int
    return _lib


def _p(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _c(a, dtype):
    return None if a is None else np.ascontiguousarray(a, dtype=dtype)


class Hypergraph:
    """Host-side hypergraph in net-CSR form, as the oracle consumes it."""

    def __init__(self, n, eptr, pins, c=None, w=None):
        self.n = int(n)
        self.eptr = _c(eptr, np.int64)
        self.pins = _c(pins, np.int32)
        self.m = int(self.eptr.shape[0] - 1)
        self.P = int(self.eptr[-1])
        self.c = _c(c, np.int32)
        self.w = _c(w, np.int32)
        self._inc = None

    def incidence(self):
        if self._inc is None:
            self._inc = incidence(self)
        return self._inc


def check_hypergraph(h):
    return _load().or_check_hypergraph(h.n, h.m, h.P, _p(h.eptr), _p(h.pins), _p(h.c),
                                       _p(h.w))


def check_partition(h, part, k):
    part = _c(part, np.int32)
    return _load().or_check_partition(h.n, _p(part), k)


def incidence(h):
    vptr = np.empty(h.n + 1, np.int64)
    vnets = np.empty(h.P, np.int32)
    _load().or_incidence(h.n, h.m, _p(h.eptr), _p(h.pins), _p(vptr), _p(vnets))
    return vptr, vnets


def pin_counts(h, part, k):
    part = _c(part, np.int32)
    phi = np.empty(h.m * k, np.int32)
    _load().or_pin_counts(h.m, _p(h.eptr), _p(h.pins), _p(part), k, _p(phi))
    return phi.reshape(h.m, k)


def connectivity(phi, k):
    phi = _c(phi, np.int32)
    m = phi.size // k
    lam = np.empty(m, np.int32)
    wk = (k + 31) // 32
    conn = np.empty(m * wk, np.uint32)
    _load().or_connectivity(m, k, _p(phi), _p(lam), _p(conn))
    return lam, conn.reshape(m, wk)


def block_weights(h, part, k):
    part = _c(part, np.int32)
    W = np.empty(k, np.int64)
    _load().or_block_weights(h.n, _p(h.c), _p(part), k, _p(W))
    return W


def km1(h, lam):
    lam = _c(lam, np.int32)
    return int(_load().or_km1(h.m, _p(h.w), _p(lam)))


def lmax(total_weight, k, eps):
    return int(_load().or_lmax(int(total_weight), int(k), float(eps)))


def total_vertex_weight(h):
    return int(h.n) if h.c is None else int(h.c.astype(np.int64).sum())


def gains(h, part, k, phi=None):
    part = _c(part, np.int32)
    if phi is None:
        phi = pin_counts(h, part, k)
    phi = _c(phi, np.int32)
    vptr, vnets = h.incidence()
    g = np.empty(h.n * k, np.int64)
    b = np.empty(h.n, np.int64)
    _load().or_gains(h.n, _p(vptr), _p(vnets), _p(h.w), _p(part), k, _p(phi), _p(g), _p(b))
    return g.reshape(h.n, k), b


def gain_cache(h, part, k, phi=None):
    """The gain cache by definition: (b[n], w(I)[n], p[n, k]), all int64."""
    part = _c(part, np.int32)
    if phi is None:
        phi = pin_counts(h, part, k)
    phi = _c(phi, np.int32)
    vptr, vnets = h.incidence()
    b = np.empty(h.n, np.int64)
    wi = np.empty(h.n, np.int64)
    p = np.empty(h.n * k, np.int64)
    _load().or_gain_cache(h.n, _p(vptr), _p(vnets), _p(h.w), _p(part), k, _p(phi), _p(b),
                          _p(wi), _p(p))
    return b, wi, p.reshape(h.n, k)


def lp_round(h, k, lmax_value, part, eligible):
    """One synchronous LP round.  Returns (new_part, next_eligible, moved, stats)."""
    part = np.array(part, dtype=np.int32, copy=True)
    elig = np.array(eligible, dtype=np.uint8, copy=True)
    moved = np.empty(h.n, np.uint8)
    st = RoundStats()
    vptr, vnets = h.incidence()
    rc = _load().or_lp_round(h.n, h.m, _p(h.eptr), _p(h.pins), _p(vptr), _p(vnets),
                             _p(h.c), _p(h.w), k, int(lmax_value), _p(part), _p(elig),
                             _p(moved), ctypes.byref(st))
    if rc != OR_OK:
        raise RuntimeError("oracle lp_round failed: %d" % rc)
    return part, elig, moved, st.as_dict()


def refine(h, k, lmax_value, rounds, part):
    """R synchronous rounds.  Returns (final_part, [stats per round], km1)."""
    part = np.array(part, dtype=np.int32, copy=True)
    stats = (RoundStats * max(1, rounds))()
    km = ctypes.c_int64(0)
    rc = _load().or_refine(h.n, h.m, _p(h.eptr), _p(h.pins), _p(h.c), _p(h.w), k,
                           int(lmax_value), rounds, _p(part), stats, ctypes.byref(km))
    if rc != OR_OK:
        raise RuntimeError("oracle refine failed: %d" % rc)
    return part, [stats[r].as_dict() for r in range(rounds)], int(km.value)


def move_gains(h, k, part, move_u, move_to):
    """Exact gains of the move sequence (move j: move_u[j] -> move_to[j]) as
    if applied in order, from the partition `part` before the sequence."""
    part = _c(part, np.int32)
    mu = _c(move_u, np.int32)
    mt = _c(move_to, np.int32)
    t = int(mu.shape[0])
    g = np.empty(max(t, 1), np.int64)
    vptr, vnets = h.incidence()
    rc = _load().or_move_gains(h.n, h.m, _p(h.eptr), _p(h.pins), _p(vptr), _p(vnets), _p(h.w),
                               k, _p(part), t, _p(mu), _p(mt), _p(g))
    if rc != OR_OK:
        raise ValueError("invalid move sequence")
    return g[:t]


def best_prefix(h, k, lmax_value, part, move_u, move_to, gains):
    """(length, total gain) of the best balanced prefix (ties: longer)."""
    part = _c(part, np.int32)
    mu = _c(move_u, np.int32)
    mt = _c(move_to, np.int32)
    g = _c(gains, np.int64)
    ln = ctypes.c_int32(0)
    bg = ctypes.c_int64(0)
    _load().or_best_prefix(h.n, _p(h.c), k, int(lmax_value), _p(part), int(mu.shape[0]),
                           _p(mu), _p(mt), _p(g), ctypes.byref(ln), ctypes.byref(bg))
    return int(ln.value), int(bg.value)


def lp_round_exact(h, k, lmax_value, part, eligible):
    """One monotone LP round.  Returns (new_part, next_eligible, moved, stats,
    number of approved moves before the prefix cut)."""
    part = np.array(part, dtype=np.int32, copy=True)
    elig = np.array(eligible, dtype=np.uint8, copy=True)
    moved = np.empty(h.n, np.uint8)
    st = RoundStats()
    napp = ctypes.c_int64(0)
    vptr, vnets = h.incidence()
    rc = _load().or_lp_round_exact(h.n, h.m, _p(h.eptr), _p(h.pins), _p(vptr), _p(vnets),
                                   _p(h.c), _p(h.w), k, int(lmax_value), _p(part), _p(elig),
                                   _p(moved), ctypes.byref(st), ctypes.byref(napp))
    if rc != OR_OK:
        raise RuntimeError("oracle lp_round_exact failed: %d" % rc)
    return part, elig, moved, st.as_dict(), int(napp.value)


def refine_exact(h, k, lmax_value, rounds, part):
    """R monotone rounds.  Returns (final_part, [stats per round], km1)."""
    part = np.array(part, dtype=np.int32, copy=True)
    stats = (RoundStats * max(1, rounds))()
    km = ctypes.c_int64(0)
    rc = _load().or_refine_exact(h.n, h.m, _p(h.eptr), _p(h.pins), _p(h.c), _p(h.w), k,
                                 int(lmax_value), rounds, _p(part), stats, ctypes.byref(km))
    if rc != OR_OK:
        raise RuntimeError("oracle refine_exact failed: %d" % rc)
    return part, [stats[r].as_dict() for r in range(rounds)], int(km.value)


def rebalance_round(h, k, lmax_value, part, eligible):
    """One rebalancing round.  Returns (new_part, eligible, moved, stats)."""
    part = np.array(part, dtype=np.int32, copy=True)
    elig = np.array(eligible, dtype=np.uint8, copy=True)
    moved = np.empty(h.n, np.uint8)
    st = RoundStats()
    vptr, vnets = h.incidence()
    rc = _load().or_rebalance_round(h.n, h.m, _p(h.eptr), _p(h.pins), _p(vptr), _p(vnets),
                                    _p(h.c), _p(h.w), k, int(lmax_value), _p(part), _p(elig),
                                    _p(moved), ctypes.byref(st))
    if rc != OR_OK:
        raise RuntimeError("oracle rebalance_round failed: %d" % rc)
    return part, elig, moved, st.as_dict()


def rebalance(h, k, lmax_value, rounds, part, eligible=None):
    """`rounds` rebalancing rounds.  Returns (part, eligible, [stats], km1)."""
    part = np.array(part, dtype=np.int32, copy=True)
    elig = (np.zeros(h.n, np.uint8) if eligible is None
            else np.array(eligible, dtype=np.uint8, copy=True))
    stats = (RoundStats * max(1, rounds))()
    km = ctypes.c_int64(0)
    rc = _load().or_rebalance(h.n, h.m, _p(h.eptr), _p(h.pins), _p(h.c), _p(h.w), k,
                              int(lmax_value), rounds, _p(part), _p(elig), stats,
                              ctypes.byref(km))
    if rc != OR_OK:
        raise RuntimeError("oracle rebalance failed: %d" % rc)
    return part, elig, [stats[r].as_dict() for r in range(rounds)], int(km.value)


def contract(h, cluster):
    """Contract the clustering.  Returns (map, coarse Hypergraph); the coarse
    hypergraph has explicit weights and may have m' = 0."""
    cl = _c(cluster, np.int32)
    n, m, P = h.n, h.m, h.P
    mp = np.empty(max(n, 1), np.int32)
    cv = np.empty(max(n, 1), np.int32)
    ce = np.empty(m + 1, np.int64)
    cpn = np.empty(max(P, 1), np.int32)
    cw = np.empty(max(m, 1), np.int32)
    sizes = np.zeros(3, np.int64)
    rc = _load().or_contract(n, m, _p(h.eptr), _p(h.pins), _p(h.c), _p(h.w), _p(cl), _p(mp),
                             _p(cv), _p(ce), _p(cpn), _p(cw), _p(sizes))
    if rc == OR_ERR_INVALID:
        raise ValueError("cluster id outside [0, n)")
    if rc != OR_OK:
        raise OverflowError("a cluster weighs 2^31 or more")
    nc, mc, pc = (int(x) for x in sizes)
    coarse = Hypergraph(nc, ce[:mc + 1].copy(), cpn[:pc].copy(), cv[:nc].copy(), cw[:mc].copy())
    return mp[:n].copy(), coarse
