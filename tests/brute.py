"""Pure-Python brute force for tiny hypergraphs, written from first principles.

This is a third, independent reading of the definitions used to pin the C
oracle.  It works with Python sets and never looks at pin-count tables:

* the connectivity set of a net is the set of blocks of its pins;
* km1 is sum over nets of (|blocks of e| - 1) * w(e);
* the gain of moving u to block i is km1(Pi) - km1(Pi with u moved to i),
  i.e. the objective delta itself, not the b(u) - p_i(u) formula.

Only for inputs with a few dozen vertices.
"""


def nets_of(eptr, pins):
    return [list(pins[eptr[e]:eptr[e + 1]]) for e in range(len(eptr) - 1)]


def blocks_of(net, part):
    return {int(part[v]) for v in net}


def pin_count(net, part, i):
    return len([v for v in net if part[v] == i])


def km1(nets, w, part):
    return sum((len(blocks_of(e, part)) - 1) * (1 if w is None else int(w[j]))
               for j, e in enumerate(nets))


def move_gain(nets, w, part, u, i):
    """Objective delta of moving u to block i (positive = km1 decreases)."""
    if part[u] == i:
        return 0
    moved = list(part)
    moved[u] = i
    return km1(nets, w, part) - km1(nets, w, moved)


def incident(nets, u):
    return [j for j, e in enumerate(nets) if u in e]


def block_weight(part, c, i):
    return sum(1 if c is None else int(c[v]) for v in range(len(part)) if part[v] == i)


def lp_round(nets, n, c, w, k, lmax, part, eligible):
    """One synchronous round: brute-force select from objective deltas, sort-based
    approval, apply, next eligible set.  Same readings as the oracle: boundary
    eligible vertices only, neighbouring blocks only, key (gain desc, block
    weight asc, block id asc), candidate if gain > 0 or gain == 0 and
    c(V_t) + c(u) < c(V_a), per-target longest prefix in (gain desc, id asc)."""
    part = list(int(x) for x in part)
    W = [block_weight(part, c, i) for i in range(k)]
    cw = (lambda v: 1) if c is None else (lambda v: int(c[v]))
    cands = []
    stats = dict(eligible=0, boundary=0, candidates=0, approved=0, moved_pins=0,
                 touched_nets=0, active_pins=0, touched_pins=0)
    for u in range(n):
        if not eligible[u]:
            continue
        stats["eligible"] += 1
        inc = incident(nets, u)
        if not any(len(blocks_of(nets[j], part)) > 1 for j in inc):
            continue
        stats["boundary"] += 1
        stats["active_pins"] += len(inc)
        a = part[u]
        neighbour_blocks = set()
        for j in inc:
            neighbour_blocks |= blocks_of(nets[j], part)
        neighbour_blocks.discard(a)
        options = []
        for i in sorted(neighbour_blocks):
            if W[i] + cw(u) > lmax:
                continue
            options.append((-move_gain(nets, w, part, u, i), W[i], i))
        if not options:
            continue
        negg, wt, t = min(options)
        g = -negg
        if g > 0 or (g == 0 and W[t] + cw(u) < W[a]):
            cands.append((t, -g, u))
    stats["candidates"] = len(cands)
    cands.sort()
    approved = []
    load = list(W)
    blocked = set()
    for t, negg, u in cands:
        if t in blocked:
            continue
        if load[t] + cw(u) > lmax:
            blocked.add(t)
            continue
        load[t] += cw(u)
        approved.append((u, t))
    before = km1(nets, w, part)
    new_part = list(part)
    moved = [0] * n
    for u, t in approved:
        new_part[u] = t
        moved[u] = 1
    stats["approved"] = len(approved)
    stats["moved_pins"] = sum(len(incident(nets, u)) for u, _ in approved)
    touched = [j for j, e in enumerate(nets) if any(moved[v] for v in e)]
    stats["touched_nets"] = len(touched)
    stats["touched_pins"] = sum(len(nets[j]) for j in touched)
    nxt = [0] * n
    for j in touched:
        for v in nets[j]:
            nxt[v] = 1
    after = km1(nets, w, new_part)
    stats["km1_delta"] = before - after
    stats["km1_after"] = after
    stats["max_block_weight"] = max(block_weight(new_part, c, i) for i in range(k))
    return new_part, nxt, moved, stats


def rebalance_round(nets, n, c, w, k, lmax, part, eligible):
    """One rebalancing round by brute force: gains as km1 deltas of single
    moves, every block a possible target.  Same readings as the oracle:
    vertices of blocks heavier than lmax are considered; target by (gain
    desc, block weight asc, block id asc) among blocks that stay <= lmax;
    per source the shortest (gain desc, id asc) prefix reaching the excess is
    proposed; per target the longest (gain desc, id asc) prefix that fits is
    applied; pins of nets with a moved vertex become eligible."""
    part = list(int(x) for x in part)
    W = [block_weight(part, c, i) for i in range(k)]
    cw = (lambda v: 1) if c is None else (lambda v: int(c[v]))
    stats = dict(eligible=0, boundary=0, candidates=0, approved=0, moved_pins=0,
                 touched_nets=0, active_pins=0, touched_pins=0)
    cands = []
    for u in range(n):
        a = part[u]
        if W[a] <= lmax:
            continue
        stats["eligible"] += 1
        stats["active_pins"] += len(incident(nets, u))
        options = [(-move_gain(nets, w, part, u, i), W[i], i) for i in range(k)
                   if i != a and W[i] + cw(u) <= lmax]
        if options:
            negg, _, t = min(options)
            cands.append((a, negg, u, t))
    stats["candidates"] = len(cands)
    proposed = []
    taken = [0] * k
    for a, negg, u, t in sorted(cands):
        if taken[a] < W[a] - lmax:
            taken[a] += cw(u)
            proposed.append((t, negg, u))
    stats["boundary"] = len(proposed)
    load = list(W)
    blocked = set()
    new_part = list(part)
    moved = [0] * n
    for t, negg, u in sorted(proposed):
        if t in blocked:
            continue
        if load[t] + cw(u) > lmax:
            blocked.add(t)
            continue
        load[t] += cw(u)
        new_part[u] = t
        moved[u] = 1
    stats["approved"] = sum(moved)
    stats["moved_pins"] = sum(len(incident(nets, u)) for u in range(n) if moved[u])
    touched = [j for j, e in enumerate(nets) if any(moved[v] for v in e)]
    stats["touched_nets"] = len(touched)
    stats["touched_pins"] = sum(len(nets[j]) for j in touched)
    nxt = [int(x) for x in eligible]
    for j in touched:
        for v in nets[j]:
            nxt[v] = 1
    before = km1(nets, w, part)
    after = km1(nets, w, new_part)
    stats["km1_delta"] = before - after
    stats["km1_after"] = after
    stats["max_block_weight"] = max(block_weight(new_part, c, i) for i in range(k))
    return new_part, nxt, moved, stats
