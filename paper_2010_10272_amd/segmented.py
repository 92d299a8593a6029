"""Many hypergraphs and their partition states in ONE device allocation.

A batch of refinements keeps every member's net CSR, incidence CSR,
workspace, partition state and round records as 256-byte aligned slices of a
single device buffer (segmented CSR: member i's arrays start at its own
offsets).  This module only plans the slices and copies the host arrays in;
loading and refinement go through the C ABI (hgref).
"""
import numpy as np
import torch

from . import hgref as H

_ALIGN = 256


class Arena:
    """Slices of one device buffer, handed out by a two-pass plan: request
    every slice first (`take`), then `allocate` once and fetch the views."""

    def __init__(self):
        self._req = []
        self._off = 0
        self.buffer = None

    def take(self, dtype, count):
        """Reserve `count` elements of `dtype`; returns a slice id."""
        nbytes = max(int(count), 1) * torch.empty((), dtype=dtype).element_size()
        self._req.append((self._off, dtype, int(count)))
        self._off += (nbytes + _ALIGN - 1) // _ALIGN * _ALIGN
        return len(self._req) - 1

    @property
    def nbytes(self):
        return self._off

    def allocate(self, device):
        self.buffer = torch.empty(max(self._off, _ALIGN), dtype=torch.uint8, device=device)

    def span(self, first, last):
        """Bytes of the buffer from slice `first` to the end of slice `last`."""
        off0 = self._req[first][0]
        off1, dtype, count = self._req[last]
        es = torch.empty((), dtype=dtype).element_size()
        return self.buffer[off0:off1 + count * es]

    def view(self, sid):
        off, dtype, count = self._req[sid]
        es = torch.empty((), dtype=dtype).element_size()
        return self.buffer[off:off + count * es].view(dtype)


def load_batch(instances, device="cuda", rounds=1, stream=None):
    """Load every instance (objects with n, eptr, pins, c, w, part, k, eps)
    into one arena and return (members, arena): hgref.Member objects whose
    graph, state and `rounds` round records all live in the arena.  All the
    partitions sit in one contiguous byte range, `arena.part_bytes`, so a
    saved copy of it restores every start partition with one copy."""
    device = torch.device(device)
    ar = Arena()
    plan = []
    # the partitions first, side by side: `part_bytes` then resets them all at once
    part_ids = [ar.take(torch.int32, int(x.n)) for x in instances]
    for x, pid in zip(instances, part_ids):
        n, m, P, k = int(x.n), int(x.eptr.shape[0] - 1), int(x.eptr[-1]), int(x.k)
        # unit weights travel as NULL (the library then reads no weight array)
        vw = None if x.c is None or bool(np.all(x.c == 1)) else x.c
        ew = None if x.w is None or bool(np.all(x.w == 1)) else x.w
        ws = H.hg_workspace_size(n, m, P, k)
        if ws == 0:
            raise H.HgError(H.HG_ERR_UNSUPPORTED, "unsupported sizes n=%d m=%d P=%d k=%d"
                            % (n, m, P, k))
        ids = {
            "eptr": ar.take(torch.int64, m + 1), "pins": ar.take(torch.int32, P),
            "vwgt": ar.take(torch.int32, n) if vw is not None else None,
            "ewgt": ar.take(torch.int32, m) if ew is not None else None,
            "vptr": ar.take(torch.int64, n + 1), "vnets": ar.take(torch.int32, P),
            "ws": ar.take(torch.uint8, ws),
            "stats": ar.take(torch.int64, max(rounds, 1) * H.STATS_WORDS),
        }
        for f, (dt, cnt) in H.state_sizes(n, m, k).items():
            ids["st_" + f] = pid if f == "part" else ar.take(dt, cnt)
        plan.append((x, n, k, ids, vw, ew))
    ar.allocate(device)
    ar.part_bytes = ar.span(part_ids[0], part_ids[-1]) if part_ids else None
    members = []
    for x, n, k, ids, vw, ew in plan:
        v = {f: (ar.view(i) if i is not None else None) for f, i in ids.items()}
        v["eptr"].copy_(torch.from_numpy(np.ascontiguousarray(x.eptr, np.int64)))
        v["pins"].copy_(torch.from_numpy(np.ascontiguousarray(x.pins, np.int32)))
        if vw is not None:
            v["vwgt"].copy_(torch.from_numpy(np.ascontiguousarray(vw, np.int32)))
        if ew is not None:
            v["ewgt"].copy_(torch.from_numpy(np.ascontiguousarray(ew, np.int32)))
        g = H.hg_load_csr(n, v["eptr"], v["pins"], v["vwgt"], v["ewgt"], k_max=k,
                          device=device, stream=stream, out=(v["vptr"], v["vnets"], v["ws"]))
        st = H.State(g, k, x.part, views={f: v["st_" + f] for f in H.STATE_FIELDS})
        v["stats"].zero_()
        members.append(H.Member(g, st, x.eps, v["stats"]))
    return members, ar
