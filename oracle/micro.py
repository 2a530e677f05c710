"""Pure-Python micro-oracle of Jet refinement -- TEST INFRASTRUCTURE ONLY.

A second, independent transcription of the refinement loop (Algorithm 3),
Jetlp with the afterburner (Algorithm 4), Jetrw (Algorithm 5) and Jetrs
(Section 4.2.2), written with Python dicts and sets for graphs of a few dozen
vertices. It is cross-checked against the C oracle iteration by iteration.

Readings shared with the C oracle (both follow the same written readings,
not each other's code): balanced <=> max part weight <= o with
o = floor((1 + lambda) W / k); argmax ties -> smallest part id; X-order ties
-> smaller vertex id; sigma = o - (0 | 1 | floor(slack/10)); eligibility
2k vw <= 3 (k w(p) - W); L' order (slot, id); evict while the weight already
evicted is below the excess; Jetrs positions by exclusive prefix over the
evicted vertices in id order; stall counts every iteration.
"""
from __future__ import annotations

M64 = (1 << 64) - 1


def mix64(z: int) -> int:
    z &= M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def neighbours(g, v):
    for e in range(int(g.xadj[v]), int(g.xadj[v + 1])):
        yield int(g.adjncy[e]), int(g.adjwgt[e])


def connectivity(g, P, v):
    """conn(v, .) as a dict part -> summed edge weight (only parts with conn > 0)."""
    c = {}
    for u, w in neighbours(g, v):
        c[P[u]] = c.get(P[u], 0) + w
    return c


def weights(g, P, k):
    w = [0] * k
    for v in range(g.n):
        w[P[v]] += int(g.vwgt[v])
    return w


def cut(g, P):
    total = 0
    for v in range(g.n):
        for u, w in neighbours(g, v):
            if P[u] != P[v]:
                total += w
    return total // 2


def limit(W, k, lambda_ppm):
    return (W * (1000000 + lambda_ppm)) // (k * 1000000)


def sigma(W, k, o, div=10):
    slack = o - (-(-W // k))
    if slack <= 0:
        return o
    if slack < div:
        return o - 1
    return o - slack // div


def slot(x):
    if x < 0:
        return 0
    if x == 0:
        return 1
    return 1 + x.bit_length()


def digest(P):
    return sum(mix64((v << 32) | p) for v, p in enumerate(P)) & M64


def jetlp(g, P, locked, c):
    cn, cd = c
    Pd, F, X = {}, {}, set()
    for v in range(g.n):
        if v in locked:
            continue
        conn = connectivity(g, P, v)
        others = [(p, x) for p, x in conn.items() if p != P[v]]
        if not others:
            continue
        top = max(x for _, x in others)
        Pd[v] = min(p for p, x in others if x == top)
        cs = conn.get(P[v], 0)
        F[v] = top - cs
        if F[v] >= 0 or -F[v] < (cn * cs) // cd:
            X.add(v)

    def before(u, v):
        return u in X and (F[u] > F[v] or (F[u] == F[v] and u < v))

    moves = {}
    for v in sorted(X):
        f2 = 0
        for u, w in neighbours(g, v):
            q = Pd[u] if before(u, v) else P[u]
            if q == Pd[v]:
                f2 += w
            elif q == P[v]:
                f2 -= w
        if f2 >= 0:
            moves[v] = Pd[v]
    return moves, len(X)


def rebalance(g, P, k, kind, lambda_ppm, level, t, seed, div=10):
    W = sum(int(x) for x in g.vwgt)
    w = weights(g, P, k)
    o = limit(W, k, lambda_ppm)
    sg = sigma(W, k, o, div)
    A = [p for p in range(k) if w[p] > o]
    B = [p for p in range(k) if w[p] <= sg]
    hseed = mix64(seed ^ ((level << 32) + t))
    loss, dest, cand = {}, {}, []
    for v in range(g.n):
        p = P[v]
        if p not in A or 2 * k * int(g.vwgt[v]) > 3 * (k * w[p] - W):
            continue
        cand.append(v)
        conn = connectivity(g, P, v)
        inB = {q: x for q, x in conn.items() if q in B}
        if kind == "RW":
            if inB:
                top = max(inB.values())
                d = min(q for q, x in inB.items() if x == top)
            else:
                h = mix64(hseed ^ v)
                d = B[(h * len(B)) >> 64]
            dest[v] = d
            loss[v] = conn.get(p, 0) - conn.get(d, 0)
        else:
            mean = sum(inB.values()) // len(inB) if inB else 0
            loss[v] = conn.get(p, 0) - mean
    evicted = []
    for p in A:
        L = sorted((slot(loss[v]), v) for v in cand if P[v] == p)
        need, s = w[p] - o, 0
        for _, v in L:
            if s >= need:
                break
            evicted.append(v)
            s += int(g.vwgt[v])
    moves = {}
    if kind == "RW":
        for v in evicted:
            moves[v] = dest[v]
    else:
        caps = [(b, sg - w[b]) for b in B]
        pos = 0
        for v in sorted(evicted):
            acc = 0
            for b, cap in caps:
                if acc <= pos < acc + cap:
                    moves[v] = b
                    break
                acc += cap
            pos += int(g.vwgt[v])
    return moves, len(cand)


def refine(g, P0, k, lambda_ppm=30000, level=0, seed=0, c=None, phi=(999, 1000), stall_limit=12,
           bmax=2, max_iters=0):
    """Returns (P_best, trace list of dicts, P_iter)."""
    if c is None:
        c = (1, 4) if level == 0 else (3, 4)
    P = [int(x) for x in P0]
    if k == 1:
        return [0] * g.n, [], [0] * g.n
    W = sum(int(x) for x in g.vwgt)
    o = limit(W, k, lambda_ppm)

    def state(P):
        w = weights(g, P, k)
        return cut(g, P), max(w)

    cur_cut, cur_max = state(P)
    best = list(P)
    bal_best = cur_max <= o
    best_cut, best_max = cur_cut, cur_max
    locked = set()
    stall = wcount = t = 0
    trace = []
    while stall < stall_limit and (max_iters <= 0 or t < max_iters):
        stall += 1
        if cur_max <= o:
            kind = "LP"
            moves, nX = jetlp(g, P, locked, c)
            locked = set(moves)
            wcount = 0
        elif wcount < bmax:
            kind = "RW"
            moves, nX = rebalance(g, P, k, "RW", lambda_ppm, level, t, seed)
            wcount += 1
        else:
            kind = "RS"
            moves, nX = rebalance(g, P, k, "RS", lambda_ppm, level, t, seed)
            wcount += 1
        for v, d in moves.items():
            P[v] = d
        cur_cut, cur_max = state(P)
        if cur_max <= o:
            if not bal_best:
                best, bal_best, best_cut, best_max, stall = list(P), True, cur_cut, cur_max, 0
            elif cur_cut < best_cut:
                if phi[1] * cur_cut < phi[0] * best_cut:
                    stall = 0
                best, best_cut, best_max = list(P), cur_cut, cur_max
        elif not bal_best and cur_max < best_max:
            best, best_max, best_cut, stall = list(P), cur_max, cur_cut, 0
        trace.append(dict(level=level, t=t, kind={"LP": 1, "RW": 2, "RS": 3}[kind], nX=nX,
                          nM=len(moves), stall=stall, wcount=wcount, balanced=int(cur_max <= o),
                          moved_w=sum(int(g.vwgt[v]) for v in moves), cut=cur_cut, maxw=cur_max,
                          best_cut=best_cut, digest=digest(P)))
        t += 1
    return best, trace, P
