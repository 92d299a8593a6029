"""Python binding of libhgref.so (include/hgref.h): argument marshalling only.

Every function keeps the name of the C entry point it calls.  Device memory
and streams come from PyTorch (ROCm builds keep the ``cuda`` device name);
all computation happens in the HIP kernels behind the C ABI.  There is no
fallback: if the shared library is missing or cannot be loaded, importing
this module raises.
"""
import ctypes
import os

import torch  # loads the HIP runtime that libhgref.so binds to

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhgref.so")   # always the in-tree build

HG_OK = 0
HG_ERR_INVALID = -1
HG_ERR_UNSUPPORTED = -2
HG_ERR_DEVICE = -3
HG_ERR_WORKSPACE = -4
HG_MAX_K = 256

STATS_FIELDS = ("eligible", "boundary", "candidates", "approved", "moved_pins", "touched_nets",
                "km1_delta", "km1_after", "max_block_weight", "km1_delta_recomputed",
                "active_pins", "touched_pins")
HG_PHASES = ("select", "approve", "finalize")
STATS_WORDS = len(STATS_FIELDS)


class HgError(RuntimeError):
    def __init__(self, code, message):
        super().__init__("hgref error %d: %s" % (code, message))
        self.code = code
        self.message = message


class GraphInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int32), ("P", ctypes.c_int64),
                ("total_vertex_weight", ctypes.c_int64), ("total_net_weight", ctypes.c_int64),
                ("max_degree", ctypes.c_int32), ("max_net_size", ctypes.c_int32),
                ("max_incident_weight", ctypes.c_int32), ("heavy_vertices", ctypes.c_int32)]


HG_SIZE_CLASSES = 4
SCHEDULE_FIELDS = ("select_chunks", "finalize_chunks", "count_chunks", "net_lanes")


class HgInstance(ctypes.Structure):
    _fields_ = [("g", ctypes.c_void_p), ("k", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("eps", ctypes.c_double), ("part", ctypes.c_void_p), ("phi", ctypes.c_void_p),
                ("netstate", ctypes.c_void_p), ("block_w", ctypes.c_void_p),
                ("eligible", ctypes.c_void_p), ("stats", ctypes.c_void_p),
                ("km1", ctypes.c_void_p)]


class HgSchedule(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int32) for f in SCHEDULE_FIELDS]


class HgRequest(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int32), ("P", ctypes.c_int64),
                ("eptr", ctypes.c_void_p), ("pins", ctypes.c_void_p), ("vwgt", ctypes.c_void_p),
                ("ewgt", ctypes.c_void_p), ("part", ctypes.c_void_p), ("k", ctypes.c_int32),
                ("rounds", ctypes.c_int32), ("eps", ctypes.c_double),
                ("part_out", ctypes.c_void_p), ("stats_out", ctypes.c_void_p),
                ("km1_out", ctypes.c_void_p), ("arrival_ms", ctypes.c_double)]


class HgRequestInfo(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("status", ctypes.c_int32),
                ("arrival_ms", ctypes.c_double), ("admit_ms", ctypes.c_double),
                ("loaded_ms", ctypes.c_double), ("done_ms", ctypes.c_double),
                ("footprint", ctypes.c_int64), ("first_step", ctypes.c_int64)]


class HgServerStats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in (
        "submitted", "completed", "failed", "steps", "member_rounds", "pin_rounds",
        "max_members", "rebuilds", "peak_bytes")]


HG_REQ_PENDING, HG_REQ_ADMITTED, HG_REQ_ACTIVE, HG_REQ_DONE = 0, 1, 2, 3


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libhgref.so not built (run __graft_entry__.build() or "
                          "python -m paper_2010_10272_amd.build): %s" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    i32, i64, vp, sz, dbl = (ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_size_t,
                             ctypes.c_double)
    lib.hg_net_words.argtypes = [i32]
    lib.hg_net_words.restype = i32
    lib.hg_netstate_words.argtypes = [i32, i32]
    lib.hg_netstate_words.restype = i64
    lib.hg_workspace_size.argtypes = [i32, i32, i64, i32]
    lib.hg_workspace_size.restype = sz
    lib.hg_load_csr.argtypes = [i32, i32, i64, vp, vp, vp, vp, vp, vp, vp, sz, i32, vp,
                                ctypes.POINTER(vp)]
    lib.hg_load_csr.restype = i32
    lib.hg_free.argtypes = [vp]
    lib.hg_free.restype = None
    lib.hg_get_info.argtypes = [vp, ctypes.POINTER(GraphInfo)]
    lib.hg_get_info.restype = i32
    lib.hg_max_block_weight.argtypes = [vp, i32, dbl]
    lib.hg_max_block_weight.restype = i64
    lib.hg_compute_pincounts.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp]
    lib.hg_compute_pincounts.restype = i32
    lib.hg_km1.argtypes = [vp, i32, vp, vp, vp]
    lib.hg_km1.restype = i32
    lib.hg_gains.argtypes = [vp, i32, vp, vp, vp, vp, vp]
    lib.hg_gains.restype = i32
    lib.hg_lp_round.argtypes = [vp, i32, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.hg_lp_round.restype = i32
    lib.hg_lp_round_noalloc.argtypes = [vp, i32, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.hg_lp_round_noalloc.restype = i32
    lib.hg_refine.argtypes = [vp, i32, dbl, i32, vp, vp, vp, vp, vp, vp, vp, i32, vp]
    lib.hg_refine.restype = i32
    lib.hg_timing_enable.argtypes = [vp, i32]
    lib.hg_timing_enable.restype = i32
    lib.hg_timing_collect.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]
    lib.hg_timing_collect.restype = i32
    lib.hg_sync_status.argtypes = [vp, vp]
    lib.hg_sync_status.restype = i32
    inst_p = ctypes.POINTER(HgInstance)
    sched_p = ctypes.POINTER(HgSchedule)
    lib.hg_batch_table_bytes.argtypes = [inst_p, i32]
    lib.hg_batch_table_bytes.restype = sz
    lib.hg_batch_create.argtypes = [inst_p, i32, sched_p, vp, sz, vp, ctypes.POINTER(vp)]
    lib.hg_batch_create.restype = i32
    lib.hg_batch_free.argtypes = [vp]
    lib.hg_batch_free.restype = None
    lib.hg_batch_start.argtypes = [vp, vp]
    lib.hg_batch_start.restype = i32
    lib.hg_batch_round.argtypes = [vp, i32, vp]
    lib.hg_batch_round.restype = i32
    lib.hg_batch_refine.argtypes = [vp, i32, i32, vp]
    lib.hg_batch_refine.restype = i32
    lib.hg_batch_autotune.argtypes = [vp, vp, i64, i32, vp, sched_p]
    lib.hg_batch_autotune.restype = i32
    lib.hg_batch_get_schedule.argtypes = [vp, sched_p]
    lib.hg_batch_get_schedule.restype = i32
    lib.hg_request_bytes.argtypes = [i32, i32, i64, i32, i32, i32, i32]
    lib.hg_request_bytes.restype = sz
    lib.hg_server_create.argtypes = [vp, sz, sz, i32, i64, sched_p, ctypes.POINTER(vp)]
    lib.hg_server_create.restype = i32
    lib.hg_server_submit.argtypes = [vp, ctypes.POINTER(HgRequest), ctypes.POINTER(i64)]
    lib.hg_server_submit.restype = i32
    lib.hg_server_now_ms.argtypes = [vp]
    lib.hg_server_now_ms.restype = dbl
    lib.hg_server_info.argtypes = [vp, i64, ctypes.POINTER(HgRequestInfo)]
    lib.hg_server_info.restype = i32
    lib.hg_server_drain.argtypes = [vp, dbl, ctypes.POINTER(i64)]
    lib.hg_server_drain.restype = i32
    lib.hg_server_get_stats.argtypes = [vp, ctypes.POINTER(HgServerStats)]
    lib.hg_server_get_stats.restype = i32
    lib.hg_server_free.argtypes = [vp]
    lib.hg_server_free.restype = None
    lib.hg_moves_workspace_size.argtypes = [i32, i32, i32]
    lib.hg_moves_workspace_size.restype = sz
    lib.hg_move_gains.argtypes = [vp, i32, vp, vp, i32, vp, vp, vp, vp, sz, vp]
    lib.hg_move_gains.restype = i32
    lib.hg_best_prefix.argtypes = [vp, i32, i64, vp, vp, i32, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.hg_best_prefix.restype = i32
    lib.hg_lp_round_exact.argtypes = [vp, i32, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.hg_lp_round_exact.restype = i32
    lib.hg_refine_exact.argtypes = [vp, i32, dbl, i32, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.hg_refine_exact.restype = i32
    lib.hg_gain_cache_bytes.argtypes = [i32, i32]
    lib.hg_gain_cache_bytes.restype = i64
    lib.hg_gain_cache_init.argtypes = [vp, i32, vp, vp, vp, vp]
    lib.hg_gain_cache_init.restype = i32
    lib.hg_lp_round_cached.argtypes = [vp, i32, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.hg_lp_round_cached.restype = i32
    lib.hg_refine_cached.argtypes = [vp, i32, dbl, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.hg_refine_cached.restype = i32
    lib.hg_rebalance_workspace_size.argtypes = [i32, i32]
    lib.hg_rebalance_workspace_size.restype = sz
    lib.hg_rebalance.argtypes = [vp, i32, i64, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.hg_rebalance.restype = i32
    lib.hg_contract_workspace_size.argtypes = [i32, i32, i64]
    lib.hg_contract_workspace_size.restype = sz
    lib.hg_contract.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.hg_contract.restype = i32
    lib.hg_last_error.argtypes = []
    lib.hg_last_error.restype = ctypes.c_char_p
    return lib


_lib = _load()


def _check(rc):
    if rc != HG_OK:
        raise HgError(rc, _lib.hg_last_error().decode(errors="replace"))


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def _dev(x, dtype, device):
    if x is None:
        return None
    if isinstance(x, torch.Tensor):
        return x.to(device=device, dtype=dtype).contiguous()
    return torch.as_tensor(x).to(device=device, dtype=dtype).contiguous()


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def hg_net_words(k):
    return int(_lib.hg_net_words(int(k)))


def hg_netstate_words(m, k):
    return int(_lib.hg_netstate_words(int(m), int(k)))


def hg_workspace_size(n, m, P, k_max):
    return int(_lib.hg_workspace_size(int(n), int(m), int(P), int(k_max)))


class Graph:
    """A loaded hypergraph: owns the device tensors the C handle borrows."""

    def __init__(self, handle, tensors, n, m, P, k_max):
        self._h = handle
        self._t = tensors
        self.n, self.m, self.P, self.k_max = n, m, P, k_max
        self.device = tensors["eptr"].device

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("graph already freed")
        return self._h

    def __getattr__(self, name):
        t = self.__dict__.get("_t")
        if t is not None and name in t:
            return t[name]
        raise AttributeError(name)

    def free(self):
        if self._h is not None:
            torch.cuda.synchronize(self.device)
            _lib.hg_free(self._h)
            self._h = None

    def __del__(self):
        try:
            if self._h is not None:
                _lib.hg_free(self._h)
                self._h = None
        except Exception:
            pass


def hg_load_csr(n, eptr, pins, vwgt=None, ewgt=None, k_max=HG_MAX_K, device="cuda",
                stream=None, out=None):
    """Load a net-CSR hypergraph (arrays or tensors) onto the device and build
    its incidence CSR.  Returns a Graph.  Synchronizes the stream.  `out` may
    supply preallocated (vptr, vnets, workspace) device tensors."""
    device = torch.device(device)
    eptr = _dev(eptr, torch.int64, device)
    pins = _dev(pins, torch.int32, device)
    vwgt = _dev(vwgt, torch.int32, device)
    ewgt = _dev(ewgt, torch.int32, device)
    m = int(eptr.numel() - 1)
    P = int(pins.numel())
    ws_bytes = hg_workspace_size(n, m, P, k_max)
    if ws_bytes == 0:
        raise HgError(HG_ERR_UNSUPPORTED, "unsupported sizes n=%d m=%d P=%d k_max=%d"
                      % (n, m, P, k_max))
    if out is not None:
        vptr, vnets, ws = out
        if vptr.numel() < n + 1 or vnets.numel() < P or ws.numel() < ws_bytes:
            raise ValueError("preallocated buffers too small")
    else:
        vptr = torch.empty(n + 1, dtype=torch.int64, device=device)
        vnets = torch.empty(max(P, 1), dtype=torch.int32, device=device)
        ws = torch.empty(ws_bytes, dtype=torch.uint8, device=device)
    h = ctypes.c_void_p()
    _check(_lib.hg_load_csr(int(n), m, P, _ptr(eptr), _ptr(pins), _ptr(vwgt), _ptr(ewgt),
                            _ptr(vptr), _ptr(vnets), _ptr(ws), ws_bytes, int(k_max),
                            _stream(stream), ctypes.byref(h)))
    tensors = dict(eptr=eptr, pins=pins, vwgt=vwgt, ewgt=ewgt, vptr=vptr, vnets=vnets,
                   workspace=ws)
    return Graph(h, tensors, int(n), m, P, int(k_max))


def hg_get_info(g):
    info = GraphInfo()
    _check(_lib.hg_get_info(g.handle, ctypes.byref(info)))
    return {f: int(getattr(info, f)) for f, _ in GraphInfo._fields_}


def hg_max_block_weight(g, k, eps):
    v = int(_lib.hg_max_block_weight(g.handle, int(k), float(eps)))
    if v < 0:
        raise HgError(HG_ERR_INVALID, "bad k or eps")
    return v


STATE_FIELDS = ("part", "phi", "netstate", "block_w", "km1", "eligible", "moved")


def state_sizes(n, m, k):
    """(dtype, element count) of every State buffer for n vertices, m nets, k."""
    return {"part": (torch.int32, n), "phi": (torch.int32, m * k),
            "netstate": (torch.int32, hg_netstate_words(m, k)), "block_w": (torch.int64, k),
            "km1": (torch.int64, 1), "eligible": (torch.uint8, n), "moved": (torch.uint8, n)}


class State:
    """Device state of one k-way partition of a graph (caller-owned buffers).

    `views` may supply every buffer (STATE_FIELDS, sized as state_sizes says),
    for example slices of one large allocation shared by many instances; the
    start partition is copied into views["part"]."""

    def __init__(self, g, k, part, views=None):
        dev = g.device
        self.k = int(k)
        sizes = state_sizes(g.n, g.m, self.k)
        if views is None:
            views = {f: torch.empty(cnt, dtype=dt, device=dev) for f, (dt, cnt) in sizes.items()}
        for f, (dt, cnt) in sizes.items():
            t = views[f]
            if t.dtype != dt or t.numel() != cnt or not t.is_contiguous():
                raise ValueError("state buffer %s must be %d contiguous %s" % (f, cnt, dt))
            setattr(self, f, t)
        self.part.copy_(_dev(part, torch.int32, dev))
        self.eligible.fill_(1)
        self.moved.zero_()


def hg_compute_pincounts(g, st, stream=None):
    _check(_lib.hg_compute_pincounts(g.handle, st.k, _ptr(st.part), _ptr(st.phi),
                                     _ptr(st.netstate), _ptr(st.block_w), _ptr(st.km1),
                                     _stream(stream)))


def hg_km1(g, k, netstate, out=None, stream=None):
    if out is None:
        out = torch.empty(1, dtype=torch.int64, device=netstate.device)
    _check(_lib.hg_km1(g.handle, int(k), _ptr(netstate), _ptr(out), _stream(stream)))
    return out


def hg_gains(g, k, part, netstate, gains=None, benefit=None, stream=None):
    dev = netstate.device
    if gains is None:
        gains = torch.empty(g.n * int(k), dtype=torch.int64, device=dev)
    _check(_lib.hg_gains(g.handle, int(k), _ptr(part), _ptr(netstate), _ptr(gains),
                         _ptr(benefit), _stream(stream)))
    return gains, benefit


def hg_lp_round(g, st, max_block_w, stats, moved=True, stream=None):
    """One label-propagation round on State st; stats: int64 device tensor of
    STATS_WORDS entries."""
    _check(_lib.hg_lp_round(g.handle, st.k, int(max_block_w), _ptr(st.part), _ptr(st.phi),
                            _ptr(st.netstate), _ptr(st.block_w), _ptr(st.eligible),
                            _ptr(st.moved) if moved else None, _ptr(st.km1), _ptr(stats),
                            _stream(stream)))


def hg_lp_round_noalloc(g, st, max_block_w, stats, moved=True, stream=None):
    """hg_lp_round with the round scratch in the library's fixed device array
    (allocates nothing; n, m <= 2^20)."""
    _check(_lib.hg_lp_round_noalloc(g.handle, st.k, int(max_block_w), _ptr(st.part),
                                    _ptr(st.phi), _ptr(st.netstate), _ptr(st.block_w),
                                    _ptr(st.eligible), _ptr(st.moved) if moved else None,
                                    _ptr(st.km1), _ptr(stats), _stream(stream)))


def hg_refine(g, st, eps, rounds, stats, use_graph=True, stream=None):
    """Pin counts from st.part, then `rounds` LP rounds; stats: int64 device
    tensor of rounds * STATS_WORDS entries."""
    _check(_lib.hg_refine(g.handle, st.k, float(eps), int(rounds), _ptr(st.part), _ptr(st.phi),
                          _ptr(st.netstate), _ptr(st.block_w), _ptr(st.eligible), _ptr(stats),
                          _ptr(st.km1), 1 if use_graph else 0, _stream(stream)))


def hg_timing_enable(g, enable=True):
    _check(_lib.hg_timing_enable(g.handle, 1 if enable else 0))


def hg_timing_collect(g):
    """Per-phase milliseconds summed over the rounds timed since the last call,
    and the number of those rounds."""
    ms = (ctypes.c_double * len(HG_PHASES))()
    rounds = ctypes.c_int64(0)
    _check(_lib.hg_timing_collect(g.handle, ms, ctypes.byref(rounds)))
    return dict(zip(HG_PHASES, list(ms))), int(rounds.value)


def hg_sync_status(g, stream=None):
    _check(_lib.hg_sync_status(g.handle, _stream(stream)))


def stats_to_dicts(stats):
    """Device stats tensor -> list of dicts (synchronizes)."""
    a = stats.view(-1, STATS_WORDS).cpu().tolist()
    return [dict(zip(STATS_FIELDS, row)) for row in a]


def decode_netstate(netstate, m, k):
    """Split a net-state tensor into (w, lambda, Lambda words, S words) views."""
    rw = hg_net_words(k)
    wk = 1
    while wk * 32 < k:
        wk *= 2
    r = netstate[:m * rw].view(m, rw)
    return r[:, 0], r[:, 1], r[:, 2:2 + wk], r[:, 2 + wk:2 + 2 * wk]


# ---------------------------------------------------------------- batches

class Member:
    """One refinement in a batch: a Graph, its State, eps and a device stats
    tensor of at least rounds * STATS_WORDS int64 entries."""

    def __init__(self, g, st, eps, stats):
        self.g, self.st, self.eps, self.stats = g, st, float(eps), stats

    def _c(self):
        st = self.st
        return HgInstance(self.g.handle.value, st.k, 0, self.eps, st.part.data_ptr(),
                          st.phi.data_ptr(), st.netstate.data_ptr(), st.block_w.data_ptr(),
                          st.eligible.data_ptr(), self.stats.data_ptr(), st.km1.data_ptr())


def _members_c(members):
    arr = (HgInstance * len(members))()
    for i, mb in enumerate(members):
        arr[i] = mb._c()
    return arr


def _schedule_c(sched):
    if sched is None:
        return None
    arr = (HgSchedule * HG_SIZE_CLASSES)()
    for c in range(HG_SIZE_CLASSES):
        for f in SCHEDULE_FIELDS:
            setattr(arr[c], f, int(sched[c][f]))
    return arr


def _schedule_py(arr):
    return [{f: int(getattr(arr[c], f)) for f in SCHEDULE_FIELDS} for c in range(HG_SIZE_CLASSES)]


class Batch:
    """A batch handle with the device table it reads and the members it
    refers to (kept alive with it)."""

    def __init__(self, handle, members, table):
        self._h = handle
        self.members = list(members)
        self.table = table

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("batch already freed")
        return self._h

    def free(self):
        if self._h is not None:
            _lib.hg_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def hg_batch_table_bytes(members):
    arr = _members_c(members)
    return int(_lib.hg_batch_table_bytes(arr, len(members)))


def hg_batch_create(members, sched=None, stream=None, table=None):
    """Members: list of Member.  sched: None or HG_SIZE_CLASSES dicts with
    SCHEDULE_FIELDS.  Returns a Batch."""
    arr = _members_c(members)
    nbytes = int(_lib.hg_batch_table_bytes(arr, len(members)))
    if nbytes == 0:
        raise HgError(HG_ERR_INVALID, _lib.hg_last_error().decode(errors="replace"))
    dev = members[0].st.part.device
    if table is None:
        table = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    h = ctypes.c_void_p()
    _check(_lib.hg_batch_create(arr, len(members), _schedule_c(sched), _ptr(table),
                                table.numel() * table.element_size(), _stream(stream),
                                ctypes.byref(h)))
    return Batch(h, members, table)


def hg_batch_start(b, stream=None):
    _check(_lib.hg_batch_start(b.handle, _stream(stream)))


def hg_batch_round(b, round_index, stream=None):
    _check(_lib.hg_batch_round(b.handle, int(round_index), _stream(stream)))


def hg_batch_refine(b, rounds, use_graph=True, stream=None):
    _check(_lib.hg_batch_refine(b.handle, int(rounds), 1 if use_graph else 0, _stream(stream)))


def hg_batch_autotune(b, repeats=3, stream=None):
    """Tune the batch's schedules in place; returns the chosen schedules."""
    total = sum(mb.g.n for mb in b.members)
    save = torch.empty(max(total, 1), dtype=torch.int32, device=b.table.device)
    out = (HgSchedule * HG_SIZE_CLASSES)()
    _check(_lib.hg_batch_autotune(b.handle, _ptr(save), total, int(repeats), _stream(stream),
                                  out))
    return _schedule_py(out)


def hg_batch_get_schedule(b=None):
    out = (HgSchedule * HG_SIZE_CLASSES)()
    _check(_lib.hg_batch_get_schedule(b.handle if b is not None else None, out))
    return _schedule_py(out)


def hg_batch_free(b):
    b.free()


# ---------------------------------------------------------------- serving

def hg_request_bytes(n, m, P, k, rounds, weighted_vertices=False, weighted_nets=False):
    return int(_lib.hg_request_bytes(int(n), int(m), int(P), int(k), int(rounds),
                                     1 if weighted_vertices else 0, 1 if weighted_nets else 0))


def _host(x, dtype):
    """A contiguous CPU tensor of `dtype` (page-locked if it already is)."""
    if x is None:
        return None
    if isinstance(x, torch.Tensor):
        t = x.to(dtype=dtype)
        if t.is_cuda:
            raise ValueError("request arrays live in host memory")
        return t.contiguous()
    return torch.as_tensor(x).to(dtype=dtype).contiguous()


class Server:
    """A request server on an arena tensor it owns (see hg_server_create).
    Jobs keep their host arrays and page-locked result buffers here until
    they are done."""

    def __init__(self, arena_bytes, table_bytes=64 << 20, max_active=256, sched=None,
                 device="cuda", big_pins=0):
        self.device = torch.device(device)
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(_lib.hg_server_create(_ptr(self.arena), int(arena_bytes), int(table_bytes),
                                         int(max_active), int(big_pins), _schedule_c(sched),
                                         ctypes.byref(h)))
        self._h = h
        self.jobs = {}

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("server already freed")
        return self._h

    def free(self, timeout_ms=120000.0):
        """Wait (up to timeout_ms) for every job, then stop the server.  Raises
        and keeps the server if jobs are still outstanding."""
        if self._h is not None:
            left = hg_server_drain(self, timeout_ms)
            if left:
                raise HgError(HG_ERR_DEVICE, "%d jobs still outstanding" % left)
            _lib.hg_server_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free(timeout_ms=0.0)
        except Exception:
            pass


def hg_server_create(arena_bytes, table_bytes=64 << 20, max_active=256, sched=None,
                     device="cuda", big_pins=0):
    return Server(arena_bytes, table_bytes, max_active, sched, device, big_pins)


def hg_server_submit(srv, n, eptr, pins, part, k, rounds, eps, vwgt=None, ewgt=None,
                     arrival_ms=None, results=True):
    """Queue one job; arrays are host arrays or CPU tensors (page-locked ones
    avoid blocking copies).  With results=True the final partition, round
    records and km1 come back into new page-locked tensors, with a tuple
    (part, stats, km1) into the caller's (see hg_server_result).  Returns the
    job id."""
    eptr = _host(eptr, torch.int64)
    pins = _host(pins, torch.int32)
    part = _host(part, torch.int32)
    vwgt = _host(vwgt, torch.int32)
    ewgt = _host(ewgt, torch.int32)
    m = int(eptr.numel() - 1)
    P = int(pins.numel())
    out = None
    if isinstance(results, (tuple, list)):
        out = tuple(results)          # caller's (part, stats, km1) host tensors
        if (out[0].numel() < int(n) or out[1].numel() < int(rounds) * STATS_WORDS
                or out[2].numel() < 1):
            raise ValueError("result buffers too small")
    elif results:
        out = (torch.empty(int(n), dtype=torch.int32, pin_memory=True),
               torch.zeros(int(rounds) * STATS_WORDS, dtype=torch.int64, pin_memory=True),
               torch.zeros(1, dtype=torch.int64, pin_memory=True))
    ptr = (lambda t: None if t is None else t.data_ptr())
    req = HgRequest(int(n), m, P, ptr(eptr), ptr(pins), ptr(vwgt), ptr(ewgt), ptr(part), int(k),
                    int(rounds), float(eps), ptr(out[0]) if out else None,
                    ptr(out[1]) if out else None, ptr(out[2]) if out else None,
                    float(arrival_ms) if arrival_ms is not None else hg_server_now_ms(srv))
    jid = ctypes.c_int64(-1)
    _check(_lib.hg_server_submit(srv.handle, ctypes.byref(req), ctypes.byref(jid)))
    srv.jobs[int(jid.value)] = (eptr, pins, part, vwgt, ewgt, out)
    return int(jid.value)


def hg_server_now_ms(srv):
    return float(_lib.hg_server_now_ms(srv.handle))


def hg_server_info(srv, jid):
    info = HgRequestInfo()
    rc = _lib.hg_server_info(srv.handle, int(jid), ctypes.byref(info))
    _check(rc)
    d = {f: getattr(info, f) for f, _ in HgRequestInfo._fields_}
    if d["status"] != HG_OK:
        d["message"] = _lib.hg_last_error().decode(errors="replace")
    return d


def hg_server_result(srv, jid):
    """(part, round records as dicts, km1) of a finished job (host tensors)."""
    out = srv.jobs[int(jid)][5]
    if out is None:
        return None
    n = srv.jobs[int(jid)][2].numel()
    return out[0][:n], stats_to_dicts(out[1]), int(out[2][0].item())


def hg_server_drain(srv, timeout_ms=-1.0):
    """Wait for every submitted job; returns how many are still outstanding."""
    left = ctypes.c_int64(0)
    _check(_lib.hg_server_drain(srv.handle, float(timeout_ms), ctypes.byref(left)))
    return int(left.value)


def hg_server_get_stats(srv):
    st = HgServerStats()
    _check(_lib.hg_server_get_stats(srv.handle, ctypes.byref(st)))
    return {f: int(getattr(st, f)) for f, _ in HgServerStats._fields_}


def hg_server_release(srv, jid):
    """Drop the host arrays and results kept for a finished job."""
    srv.jobs.pop(int(jid), None)


def hg_server_free(srv):
    srv.free()


# ---------------------------------------------------------------- move sequences

def hg_moves_workspace_size(n, m, k):
    return int(_lib.hg_moves_workspace_size(int(n), int(m), int(k)))


def moves_workspace(g, k):
    """A device workspace tensor for the move-sequence calls on graph g."""
    nbytes = hg_moves_workspace_size(g.n, g.m, k)
    if nbytes == 0:
        raise HgError(HG_ERR_UNSUPPORTED, "unsupported sizes")
    return torch.empty(nbytes, dtype=torch.uint8, device=g.device)


def hg_move_gains(g, k, part, phi, move_u, move_to, ws, gains=None, stream=None):
    dev = g.device
    move_u = _dev(move_u, torch.int32, dev)
    move_to = _dev(move_to, torch.int32, dev)
    t = int(move_u.numel())
    if gains is None:
        gains = torch.empty(max(t, 1), dtype=torch.int64, device=dev)
    _check(_lib.hg_move_gains(g.handle, int(k), _ptr(part), _ptr(phi), t, _ptr(move_u),
                              _ptr(move_to), _ptr(gains), _ptr(ws), ws.numel(), _stream(stream)))
    return gains[:t]


def hg_best_prefix(g, k, max_block_w, part, block_w, move_u, move_to, gains, ws, stream=None):
    """(best_len, best_gain) as device tensors of one element."""
    dev = g.device
    move_u = _dev(move_u, torch.int32, dev)
    move_to = _dev(move_to, torch.int32, dev)
    gains = _dev(gains, torch.int64, dev)
    t = int(move_u.numel())
    blen = torch.zeros(1, dtype=torch.int32, device=dev)
    bgain = torch.zeros(1, dtype=torch.int64, device=dev)
    _check(_lib.hg_best_prefix(g.handle, int(k), int(max_block_w), _ptr(part), _ptr(block_w), t,
                               _ptr(move_u) if t else None, _ptr(move_to) if t else None,
                               _ptr(gains) if t else None, _ptr(blen), _ptr(bgain), _ptr(ws),
                               ws.numel(), _stream(stream)))
    return blen, bgain


def hg_lp_round_exact(g, st, max_block_w, stats, ws, moved=True, stream=None):
    _check(_lib.hg_lp_round_exact(g.handle, st.k, int(max_block_w), _ptr(st.part), _ptr(st.phi),
                                  _ptr(st.netstate), _ptr(st.block_w), _ptr(st.eligible),
                                  _ptr(st.moved) if moved else None, _ptr(st.km1), _ptr(stats),
                                  _ptr(ws), ws.numel(), _stream(stream)))


def hg_refine_exact(g, st, eps, rounds, stats, ws, stream=None):
    _check(_lib.hg_refine_exact(g.handle, st.k, float(eps), int(rounds), _ptr(st.part),
                                _ptr(st.phi), _ptr(st.netstate), _ptr(st.block_w),
                                _ptr(st.eligible), _ptr(stats), _ptr(st.km1), _ptr(ws),
                                ws.numel(), _stream(stream)))


# ---------------------------------------------------------------- gain cache

def gain_cache(g, k):
    """A device buffer for the gain cache of g at k blocks (int32, 16-byte
    aligned as every torch allocation is)."""
    nbytes = int(_lib.hg_gain_cache_bytes(g.n, int(k)))
    if nbytes < 0:
        raise ValueError("bad n or k for a gain cache")
    return torch.empty(nbytes // 4, dtype=torch.int32, device=g.device)


def cache_views(g, k, cache):
    """(b[n], w(I)[n], p[n, k]) views of a gain-cache buffer."""
    n, k = g.n, int(k)
    pbase = (2 * n + 3) & ~3
    ks = (k + 3) & ~3
    return cache[:n], cache[n:2 * n], cache[pbase:pbase + n * ks].view(n, ks)[:, :k]


def hg_gain_cache_init(g, k, part, netstate, cache, stream=None):
    _check(_lib.hg_gain_cache_init(g.handle, int(k), _ptr(part), _ptr(netstate), _ptr(cache),
                                   _stream(stream)))


def hg_lp_round_cached(g, st, max_block_w, stats, cache, stream=None):
    _check(_lib.hg_lp_round_cached(g.handle, st.k, int(max_block_w), _ptr(st.part),
                                   _ptr(st.phi), _ptr(st.netstate), _ptr(st.block_w),
                                   _ptr(st.eligible), _ptr(st.moved), _ptr(st.km1), _ptr(stats),
                                   _ptr(cache), _stream(stream)))


def hg_refine_cached(g, st, eps, rounds, stats, cache, stream=None):
    _check(_lib.hg_refine_cached(g.handle, st.k, float(eps), int(rounds), _ptr(st.part),
                                 _ptr(st.phi), _ptr(st.netstate), _ptr(st.block_w),
                                 _ptr(st.eligible), _ptr(st.moved), _ptr(stats), _ptr(st.km1),
                                 _ptr(cache), _stream(stream)))


# ---------------------------------------------------------------- rebalancing

def rebalance_workspace(g, k):
    nbytes = int(_lib.hg_rebalance_workspace_size(g.n, int(k)))
    if nbytes == 0:
        raise ValueError("bad n or k for a rebalance workspace")
    return torch.empty(nbytes, dtype=torch.uint8, device=g.device)


def hg_rebalance(g, st, max_block_w, rounds, stats, ws, stream=None):
    """`rounds` rebalancing rounds on State st (its pin counts must describe
    st.part); stats: int64 device tensor of rounds * STATS_WORDS entries."""
    _check(_lib.hg_rebalance(g.handle, st.k, int(max_block_w), int(rounds), _ptr(st.part),
                             _ptr(st.phi), _ptr(st.netstate), _ptr(st.block_w),
                             _ptr(st.eligible), _ptr(st.moved), _ptr(st.km1), _ptr(stats),
                             _ptr(ws), ws.numel(), _stream(stream)))


# ---------------------------------------------------------------- contraction

class Coarse:
    """Outputs of hg_contract (device tensors at their capacities) and the
    coarse sizes n', m', P' (read back, which synchronizes)."""

    def __init__(self, g):
        dev = g.device
        self.map = torch.empty(g.n, dtype=torch.int32, device=dev)
        self.cvwgt = torch.empty(g.n, dtype=torch.int32, device=dev)
        self.ceptr = torch.empty(g.m + 1, dtype=torch.int64, device=dev)
        self.cpins = torch.empty(g.P, dtype=torch.int32, device=dev)
        self.cewgt = torch.empty(g.m, dtype=torch.int32, device=dev)
        self.sizes = torch.zeros(3, dtype=torch.int64, device=dev)

    def read_sizes(self):
        return tuple(int(x) for x in self.sizes.cpu().tolist())

    def views(self):
        """(map, cvwgt, ceptr, cpins, cewgt) cut to the coarse sizes."""
        nc, mc, pc = self.read_sizes()
        return (self.map, self.cvwgt[:nc], self.ceptr[:mc + 1], self.cpins[:pc],
                self.cewgt[:mc])


def contract_workspace(g):
    nbytes = int(_lib.hg_contract_workspace_size(g.n, g.m, g.P))
    if nbytes == 0:
        raise ValueError("bad sizes for a contraction workspace")
    return torch.empty(nbytes, dtype=torch.uint8, device=g.device)


def hg_contract(g, cluster, out, ws, stream=None):
    cluster = _dev(cluster, torch.int32, g.device)
    out.cluster = cluster          # alive while the call may still be running
    _check(_lib.hg_contract(g.handle, _ptr(cluster), _ptr(out.map), _ptr(out.cvwgt),
                            _ptr(out.ceptr), _ptr(out.cpins), _ptr(out.cewgt), _ptr(out.sizes),
                            _ptr(ws), ws.numel(), _stream(stream)))
    return out
