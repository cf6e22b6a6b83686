"""O6: contraction-path cost model, greedy and randomised-greedy search, and
index slicing (Sec. 3.1: Flop-minimising pairwise order, slicing of indices
into independent sub-networks).

The paper states the goal (a pseudo-optimal pairwise order found quickly,
then slicing to bound intermediate memory) but not the heuristics.  This
module fixes one reading, and the native planner implements the same
reading independently; the tests require both to produce the same path,
cost and slice set.

Cost model, evaluated in IEEE double arithmetic in exactly this order
    size(S)   = product of extents over S, labels in ascending order
    flops     = 8 * size(A u B) per step (one complex multiply-add = 8 real
                flops), summed over steps in path order
    result    = labels of A u B that are open or still held by another live
                tensor (ascending)
    peak      = max over steps of [sum of sizes of all live tensors before the
                step + size(C) + size(A) + size(B)]; the second A and B terms
                reserve room for permuted copies.  Bytes = 8 * peak (complex64).
Greedy step
    candidates: pairs of live tensors sharing a label (all pairs if none do);
    choose the minimum of (size(C) - size(A) - size(B), flops, i, j), i < j.
Randomised greedy
    sigma = sign(d) * log2(1 + |d|) with d as above; candidate c is drawn with
    weight exp(-(sigma_c - sigma_min) / T), candidates in (i, j) order, using
    SplitMix64 (Steele, Lea, Flood 2014): state += 0x9E3779B97F4A7C15, then
    the published mixing steps; a uniform is (z >> 11) * 2^-53.  Trial r
    seeds its own state with the first output of a generator started at
    seed + r * 0x9E3779B97F4A7C15.  The deterministic greedy path is trial
    -1; the best trial by (flops, peak) wins, earlier trials on ties.
Slicing
    while 8 * peak > budget: among non-open, not yet sliced labels of A, B
    and C at the first step attaining the peak, slice the one giving the
    smallest (peak, total flops over all slices, label).

Recursive bisection (Sec. 3.1 names graph partitioning "plus heuristics";
this is one reading of that, not the paper's partitioner)
    leaf graph: one edge per label held by exactly two leaves (open labels
    excluded); adjacency lists filled in ascending label order.  A trial
    draws eps = 0.05 + 0.85 u, then cutoff = (2, 4, 8, 16, 32)[x mod 5] from
    its stream.  A node set of one leaf is that leaf; a set of at most
    `cutoff` leaves is ordered by greedy with the labels it shares with the
    rest of the network kept open; a larger set is bisected and its halves'
    trees are contracted last.  Bisection: part 0 starts at the leaf
    nodes[x mod n] and grows, one leaf at a time up to floor(n/2), by the
    outside leaf with most adjacency entries into part 0 (ties: smallest id;
    none adjacent: smallest outside id).  Then Fiduccia-Mattheyses passes
    (at most 6): repeatedly move the unlocked leaf of largest cut gain (ties:
    smallest id) whose move keeps both parts within [lo, n - lo], lo =
    max(1, floor((1 - eps) n / 2)); keep the shortest prefix of moves with
    the lowest cut; stop when a pass does not lower the cut.  Each split
    runs this 8 times (the seed leaf drawn anew each time) and keeps the
    lowest final cut, the first on ties.  Each tree is then reconfigured:
    for every internal node in creation order, the frontier of its subtree
    grows to at most 8 tensors by expanding the internal frontier node of
    largest result size (ties: smallest id); the cheapest pairwise order of
    that frontier (exact search over subsets, the lowest-bit subset of a
    split first, splits in descending subset order, strict improvement;
    kept labels = the node's result) replaces the subtree when it costs
    strictly fewer flops, the freed internal ids reused in ascending order in
    post-order; passes repeat (at most 8) until one no longer lowers the
    tree's flops.  The plain greedy
    path and every trial are sliced to the budget, and the lowest (total
    flops, peak, index) wins.

Parity pins (tests): hand-computed costs of small paths; greedy never worse
than... (none; greedy is a heuristic) -- instead an exhaustive search over
all pairwise orders on <= 7 tensors bounds it from below; sliced peak <=
budget; slicing invariance of the contracted value (with O2).
"""

from __future__ import annotations

import math
from typing import Dict, Iterable, List, Sequence, Tuple

MASK64 = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15


class SplitMix64:
    def __init__(self, state: int):
        self.state = state & MASK64

    def next_u64(self) -> int:
        self.state = (self.state + GOLDEN) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def uniform(self) -> float:
        return (self.next_u64() >> 11) * (1.0 / 9007199254740992.0)


def size_of(labels: Iterable[int], ext: Dict[int, int]) -> float:
    s = 1.0
    for l in sorted(labels):
        s = s * float(ext[l])
    return s


class _State:
    def __init__(self, leaves: Sequence[Iterable[int]], open_set, sliced):
        self.sets = {i: frozenset(l for l in ls if l not in sliced) for i, ls in enumerate(leaves)}
        self.open = frozenset(open_set)
        self.count: Dict[int, int] = {}
        for s in self.sets.values():
            for l in s:
                self.count[l] = self.count.get(l, 0) + 1
        self.next_id = len(leaves)

    def result(self, i: int, j: int) -> frozenset:
        a, b = self.sets[i], self.sets[j]
        out = []
        for l in a | b:
            other = self.count[l] - (l in a) - (l in b)
            if l in self.open or other > 0:
                out.append(l)
        return frozenset(out)

    def merge(self, i: int, j: int) -> Tuple[frozenset, frozenset, frozenset, int]:
        a, b = self.sets.pop(i), self.sets.pop(j)
        for l in a:
            self.count[l] -= 1
        for l in b:
            self.count[l] -= 1
        c = []
        for l in a | b:
            if l in self.open or self.count[l] > 0:
                c.append(l)
        c = frozenset(c)
        for l in c:
            self.count[l] = self.count.get(l, 0) + 1
        nid = self.next_id
        self.sets[nid] = c
        self.next_id += 1
        return a, b, c, nid

    def candidates(self) -> List[Tuple[int, int]]:
        by_label: Dict[int, List[int]] = {}
        for i, s in self.sets.items():
            for l in s:
                by_label.setdefault(l, []).append(i)
        pairs = set()
        for ids in by_label.values():
            ids = sorted(ids)
            for x in range(len(ids)):
                for y in range(x + 1, len(ids)):
                    pairs.add((ids[x], ids[y]))
        if not pairs:
            ids = sorted(self.sets)
            pairs = {(ids[x], ids[y]) for x in range(len(ids)) for y in range(x + 1, len(ids))}
        return sorted(pairs)


def _score(st: _State, i: int, j: int, ext) -> Tuple[float, float]:
    c = st.result(i, j)
    d = size_of(c, ext) - size_of(st.sets[i], ext) - size_of(st.sets[j], ext)
    fl = 8.0 * size_of(st.sets[i] | st.sets[j], ext)
    return d, fl


def greedy_path(leaves, ext, open_set=(), rng: SplitMix64 | None = None,
                temperature: float = 1.0) -> List[Tuple[int, int]]:
    """Deterministic greedy (rng None) or one randomised-greedy trial."""
    st = _State(leaves, open_set, ())
    path = []
    while len(st.sets) > 1:
        cands = st.candidates()
        scored = [(_score(st, i, j, ext), i, j) for (i, j) in cands]
        if rng is None:
            (d, fl), i, j = min(scored, key=lambda x: (x[0][0], x[0][1], x[1], x[2]))
        else:
            sig = [math.copysign(math.log2(1.0 + abs(s[0][0])), s[0][0]) for s in scored]
            smin = min(sig)
            w = [math.exp(-(s - smin) / temperature) for s in sig]
            tot = 0.0
            for x in w:
                tot += x
            u = rng.uniform() * tot
            acc = 0.0
            pick = len(w) - 1
            for k, x in enumerate(w):
                acc += x
                if acc >= u:
                    pick = k
                    break
            _, i, j = scored[pick]
        st.merge(i, j)
        path.append((i, j))
    return path


def path_stats(leaves, ext, path, open_set=(), sliced=()) -> dict:
    """Per-slice flops, peak live elements and per-step label sets."""
    st = _State(leaves, open_set, set(sliced))
    live = 0.0
    for s in st.sets.values():
        live += size_of(s, ext)
    flops = 0.0
    peak = 0.0
    peak_step = -1
    steps = []
    for t, (i, j) in enumerate(path):
        sa, sb = st.sets[i], st.sets[j]
        c = st.result(i, j)
        szA, szB, szC = size_of(sa, ext), size_of(sb, ext), size_of(c, ext)
        p = live + szC + szA + szB
        if p > peak:
            peak, peak_step = p, t
        flops += 8.0 * size_of(sa | sb, ext)
        a, b, c2, _ = st.merge(i, j)
        assert c2 == c
        live = live - szA - szB + szC
        steps.append((sa, sb, c))
    n_slices = 1.0
    for l in sorted(sliced):
        n_slices *= float(ext[l])
    return {"flops": flops, "peak": peak, "peak_step": peak_step, "steps": steps,
            "n_slices": n_slices, "total_flops": flops * n_slices}


RERANK = 16   # candidates re-ranked by their sliced cost when a budget is given


def random_greedy_path(leaves, ext, open_set=(), seed: int = 0, trials: int = 32,
                       temperature: float = 1.0, budget_bytes: float = 0.0):
    """Best of the plain greedy path and `trials` randomised ones (trial r
    draws from SplitMix64 seeded with seed + r * golden ratio), by unsliced
    (flops, peak), earlier candidates winning ties.  With a memory budget,
    the RERANK best are sliced to it (slice_path) and the lowest (total
    flops, peak) wins instead."""
    cands = [greedy_path(leaves, ext, open_set)]
    for r in range(trials):
        g = SplitMix64((seed + r * GOLDEN) & MASK64)
        rng = SplitMix64(g.next_u64())
        cands.append(greedy_path(leaves, ext, open_set, rng=rng, temperature=temperature))
    keys = []
    for i, p in enumerate(cands):
        s = path_stats(leaves, ext, p, open_set)
        keys.append((s["flops"], s["peak"], i))
    order = [k[2] for k in sorted(keys)]
    if budget_bytes <= 0:
        return cands[order[0]]
    best = None
    for rank, i in enumerate(order[:RERANK]):
        try:
            sl = slice_path(leaves, ext, cands[i], open_set, budget_bytes)
        except ValueError:
            continue
        s = path_stats(leaves, ext, cands[i], open_set, sl)
        key = (s["total_flops"], s["peak"], rank)
        if best is None or key < best[0]:
            best = (key, i)
    return cands[order[0] if best is None else best[1]]


def slice_path(leaves, ext, path, open_set, budget_bytes: float) -> List[int]:
    """Labels to slice so that 8 * peak <= budget (empty list if it fits)."""
    sliced: List[int] = []
    cur = path_stats(leaves, ext, path, open_set, sliced)
    while 8.0 * cur["peak"] > budget_bytes:
        sa, sb, sc = cur["steps"][cur["peak_step"]]
        cands = sorted(l for l in (sa | sb | sc) if l not in open_set and l not in sliced)
        if not cands:
            raise ValueError("memory budget cannot be met by slicing")
        best = None
        for l in cands:
            s = path_stats(leaves, ext, path, open_set, sliced + [l])
            key = (s["peak"], s["total_flops"], l)
            if best is None or key < best[0]:
                best = (key, l, s)
        sliced.append(best[1])
        cur = best[2]
    return sliced


# ---------------------------------------------------------------- bisection

CUTOFFS = (2, 4, 8, 16, 32)
RESTARTS = 8   # bisections tried per split, the lowest cut kept
RECONF = 8     # frontier size of the subtree reconfiguration
RECONF_PASSES = 8   # reconfiguration passes, until one no longer lowers the flops


def _leaf_graph(leaves, n_labels, open_set):
    holders = [[] for _ in range(n_labels)]
    for i, ls in enumerate(leaves):
        for l in sorted(ls):
            holders[l].append(i)
    adj = [[] for _ in leaves]
    for l in range(n_labels):
        h = holders[l]
        if len(h) == 2 and l not in open_set:
            adj[h[0]].append(h[1])
            adj[h[1]].append(h[0])
    return adj, holders


def _bisect(adj, nodes, eps, rng, side):
    """The lowest cut of RESTARTS bisections (each from its own seed leaf;
    the first on ties)."""
    best = None
    for _ in range(RESTARTS):
        p0, p1, cut = _bisect_once(adj, nodes, eps, rng, side)
        if best is None or cut < best[2]:
            best = (p0, p1, cut)
    return best[0], best[1]


def _bisect_once(adj, nodes, eps, rng, side):
    n = len(nodes)
    aux = {}
    for v in nodes:
        side[v] = 1
        aux[v] = 0

    def add0(v):
        side[v] = 0
        for u in adj[v]:
            if side[u] >= 0:
                aux[u] += 1

    add0(nodes[rng.next_u64() % n])
    for _ in range(1, n // 2):
        pick = None
        for v in nodes:
            if side[v] == 1 and aux[v] > 0 and (pick is None or aux[v] > aux[pick]):
                pick = v
        if pick is None:
            pick = next(v for v in nodes if side[v] == 1)
        add0(pick)
    lo = max(1, int(math.floor((1.0 - eps) * n / 2.0)))
    hi = n - lo
    cut = sum(1 for v in nodes for u in adj[v] if side[u] >= 0 and side[u] != side[v]) // 2
    for _ in range(6):
        sizes = [0, 0]
        locked = {}
        for v in nodes:
            sizes[side[v]] += 1
            locked[v] = False
            aux[v] = sum((1 if side[u] != side[v] else -1) for u in adj[v] if side[u] >= 0)
        cur = best_c = cut
        best_k = 0
        moved = []
        for k in range(n):
            pick = None
            for v in nodes:
                if locked[v] or sizes[side[v]] - 1 < lo or sizes[1 - side[v]] + 1 > hi:
                    continue
                if pick is None or aux[v] > aux[pick]:
                    pick = v
            if pick is None:
                break
            s0 = side[pick]
            side[pick] = 1 - s0
            sizes[s0] -= 1
            sizes[1 - s0] += 1
            cur -= aux[pick]
            aux[pick] = -aux[pick]
            locked[pick] = True
            moved.append(pick)
            for u in adj[pick]:
                if side[u] >= 0:
                    aux[u] += 2 if side[u] == s0 else -2
            if cur < best_c:
                best_c, best_k = cur, k + 1
        for v in reversed(moved[best_k:]):
            side[v] = 1 - side[v]
        if best_c >= cut:
            break
        cut = best_c
    p0 = [v for v in nodes if side[v] == 0]
    p1 = [v for v in nodes if side[v] == 1]
    for v in nodes:
        side[v] = -1
    return p0, p1, cut


def partition_path(leaves, ext, open_set, rng: SplitMix64) -> List[Tuple[int, int]]:
    """One recursive-bisection contraction tree (SSA pairs)."""
    eps = 0.05 + 0.85 * rng.uniform()
    cutoff = CUTOFFS[rng.next_u64() % 5]
    n = len(leaves)
    if n <= 1:
        return []
    open_set = set(open_set)
    adj, holders = _leaf_graph(leaves, len(ext), open_set)
    side = [-1] * n
    pairs: List[Tuple[int, int]] = []
    nxt = [n]

    def build(nodes):
        if len(nodes) == 1:
            return nodes[0]
        if len(nodes) <= cutoff:
            inset = set(nodes)
            keep = set(open_set)
            for v in nodes:
                for l in leaves[v]:
                    if any(h not in inset for h in holders[l]):
                        keep.add(l)
            gp = greedy_path([leaves[v] for v in nodes], ext, keep)
            ids = list(nodes)
            for (i, j) in gp:
                pairs.append((ids[i], ids[j]))
                ids.append(nxt[0])
                nxt[0] += 1
            return ids[-1]
        p0, p1 = _bisect(adj, nodes, eps, rng, side)
        a = build(p0)
        b = build(p1)
        pairs.append((a, b))
        nxt[0] += 1
        return nxt[0] - 1

    build(list(range(n)))
    return pairs


def reconfigure_path(leaves, ext, open_set, path) -> List[Tuple[int, int]]:
    """Subtree reconfiguration of a complete SSA path (see the header)."""
    open_set = set(open_set)
    n = len(leaves)
    total = n + len(path)
    ca, cb = [-1] * total, [-1] * total
    for t, (i, j) in enumerate(path):
        ca[n + t], cb[n + t] = i, j
    holders: Dict[int, int] = {}
    for ls in leaves:
        for l in ls:
            holders[l] = holders.get(l, 0) + 1
    cnt: List[Dict[int, int]] = [dict() for _ in range(total)]
    sets: List[List[int]] = [[] for _ in range(total)]
    for i in range(n):
        for l in leaves[i]:
            cnt[i][l] = 1
        sets[i] = sorted(leaves[i])
    for v in range(n, total):
        c = dict(cnt[ca[v]])
        for l, k in cnt[cb[v]].items():
            c[l] = c.get(l, 0) + k
        cnt[v] = c
        sets[v] = sorted(l for l, k in c.items() if l in open_set or k < holders[l])

    def flops_of(a, b):
        return 8.0 * size_of(set(a) | set(b), ext)

    cost = [0.0] * total
    for v in range(n, total):
        cost[v] = flops_of(sets[ca[v]], sets[cb[v]])
    for v in range(n, total):
        F = [ca[v], cb[v]]
        region = [v]
        while len(F) < RECONF:
            pick = None
            for k, u in enumerate(F):
                if u < n:
                    continue
                su = size_of(sets[u], ext)
                if pick is None or su > size_of(sets[F[pick]], ext) or \
                        (su == size_of(sets[F[pick]], ext) and u < F[pick]):
                    pick = k
            if pick is None:
                break
            u = F[pick]
            region.append(u)
            del F[pick]
            F.append(ca[u])
            F.append(cb[u])
        if len(F) < 3:
            continue
        cur = 0.0
        for u in region:
            cur += cost[u]
        m = len(F)
        full = (1 << m) - 1
        keep_v = set(sets[v])
        rs: List[List[int]] = [[] for _ in range(full + 1)]
        for S in range(1, full + 1):
            if S & (S - 1) == 0:
                rs[S] = sets[F[(S & -S).bit_length() - 1]]
                continue
            u_set, out_set = set(), set()
            for k in range(m):
                (u_set if S >> k & 1 else out_set).update(sets[F[k]])
            rs[S] = sorted(l for l in u_set if l in keep_v or l in out_set)
        best = [0.0] * (full + 1)
        split = [0] * (full + 1)
        for S in range(1, full + 1):
            if S & (S - 1) == 0:
                continue
            low = S & -S
            bv, bs = -1.0, 0
            A = (S - 1) & S
            while A > 0:
                if A & low:
                    B = S ^ A
                    c = best[A] + best[B] + flops_of(rs[A], rs[B])
                    if bv < 0 or c < bv:
                        bv, bs = c, A
                A = (A - 1) & S
            best[S], split[S] = bv, bs
        if not best[full] < cur:
            continue
        ids = [region[0]] + sorted(region[1:])
        nxt = [1]

        def make(S):
            if S & (S - 1) == 0:
                return F[(S & -S).bit_length() - 1]
            A = split[S]
            x = make(A)
            y = make(S ^ A)
            if S == full:
                node = v
            else:
                node = ids[nxt[0]]
                nxt[0] += 1
            ca[node], cb[node] = x, y
            sets[node] = rs[S]
            cost[node] = flops_of(sets[x], sets[y])
            return node

        make(full)
    out: List[Tuple[int, int]] = []
    nid = [n]

    def emit(u):
        if u < n:
            return u
        x = emit(ca[u])
        y = emit(cb[u])
        out.append((x, y))
        nid[0] += 1
        return nid[0] - 1

    emit(total - 1)
    return out


def partition_search(leaves, ext, open_set=(), seed: int = 0, trials: int = 32,
                     budget_bytes: float = 0.0) -> List[Tuple[int, int]]:
    """Best of the plain greedy path and `trials` bisection trees by sliced
    (total flops, peak), earlier candidates winning ties."""
    cands = [greedy_path(leaves, ext, open_set)]
    for r in range(trials):
        g = SplitMix64((seed + r * GOLDEN) & MASK64)
        cur = partition_path(leaves, ext, open_set, SplitMix64(g.next_u64()))
        fl = path_stats(leaves, ext, cur, open_set)["flops"]
        for _ in range(RECONF_PASSES):
            nxt = reconfigure_path(leaves, ext, open_set, cur)
            f2 = path_stats(leaves, ext, nxt, open_set)["flops"]
            cur = nxt
            if not f2 < fl:
                break
            fl = f2
        cands.append(cur)
    best = None
    for i, p in enumerate(cands):
        try:
            sl = slice_path(leaves, ext, p, open_set, budget_bytes) if budget_bytes > 0 else []
        except ValueError:
            continue
        s = path_stats(leaves, ext, p, open_set, sl)
        key = (s["total_flops"], s["peak"], i)
        if best is None or key < best[0]:
            best = (key, i)
    return cands[0 if best is None else best[1]]
