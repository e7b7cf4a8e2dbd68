"""Exact references written independently of the oracle (test helpers).

* ``brute``: enumerate all 2^m arc states in plain integer order, decide
  s-t connectivity with a union-find (not a layered search), and add exact
  rational products with ``fractions.Fraction`` (each float p converted
  exactly).  No rounding at all.
* ``factoring``: the factoring theorem R(G) = p_e R(G / e) + (1 - p_e)
  R(G - e), recursing on contracted / deleted graphs, again in exact
  rationals.  A different algorithm from enumeration.
"""
from fractions import Fraction


def _find(par, a):
    while par[a] != a:
        par[a] = par[par[a]]
        a = par[a]
    return a


def connected_uf(n, arcs, s, t, x):
    par = list(range(n))
    for (u, v), xi in zip(arcs, x):
        if xi:
            ru, rv = _find(par, u), _find(par, v)
            if ru != rv:
                par[ru] = rv
    return _find(par, s) == _find(par, t)


def reach_directed(n, arcs, s, t, x):
    seen = {s}
    stack = [s]
    while stack:
        u = stack.pop()
        for (a, b), xi in zip(arcs, x):
            if xi and a == u and b not in seen:
                seen.add(b)
                stack.append(b)
    return t in seen


def brute(n, arcs, p, s, t, directed=False):
    """Exact (R, count, U, T1, T0) as Fractions / ints."""
    arcs = [(int(a), int(b)) for a, b in arcs]
    m = len(arcs)
    P = [Fraction(float(x)) for x in p]
    R = Fraction(0)
    U = Fraction(0)
    cnt = 0
    T1 = [Fraction(0)] * m
    T0 = [Fraction(0)] * m
    for c in range(1 << m):
        x = [(c >> i) & 1 for i in range(m)]
        q = [P[i] if x[i] else 1 - P[i] for i in range(m)]
        w = Fraction(1)
        for v in q:
            w *= v
        ok = reach_directed(n, arcs, s, t, x) if directed else connected_uf(n, arcs, s, t, x)
        if ok:
            cnt += 1
            R += w
            for i in range(m):
                wi = Fraction(1)
                for j in range(m):
                    if j != i:
                        wi *= q[j]
                if x[i]:
                    T1[i] += wi
                else:
                    T0[i] += wi
        else:
            U += w
    return R, cnt, U, T1, T0


def factoring(n, arcs, p, s, t):
    """Exact R by the factoring theorem (undirected)."""
    P = [Fraction(float(x)) for x in p]

    def rec(arcs_, probs, s_, t_):
        if s_ == t_:
            return Fraction(1)
        if not arcs_:
            return Fraction(0)
        (u, v), pe = arcs_[0], probs[0]
        rest, rp = arcs_[1:], probs[1:]
        # delete e
        r_del = rec(rest, rp, s_, t_)
        if u == v:
            return r_del
        # contract e: rename v -> u
        ren = lambda a: u if a == v else a
        r_con = rec([(ren(a), ren(b)) for a, b in rest], rp, ren(s_), ren(t_))
        return pe * r_con + (1 - pe) * r_del

    return rec([(int(a), int(b)) for a, b in arcs], P, s, t)


def layered_search_work(n, arcs, s, t, x, directed=False):
    """The layered search of Section 3.2 written out on node sets, with its
    work: (connected, layers built, arc inspections).

    Layer 1 is {s}.  Expanding a layer looks at every arc end at each of its
    nodes (working or not: the state is what the look reads), and the next
    layer is the set of nodes not in any earlier layer reached over a
    working arc.  The search stops when a layer comes out empty (layers =
    the non-empty ones) or holds t (layers = t's layer index).  A self-loop
    is one arc end at its node; an undirected arc is an end at each of its
    two nodes, a directed one only at its tail.
    """
    ends = {v: [] for v in range(n)}
    for i, (a, b) in enumerate(arcs):
        a, b = int(a), int(b)
        ends[a].append((i, b))
        if not directed and a != b:
            ends[b].append((i, a))
    placed = {s}
    layer = {s}
    built = 1
    looks = 0
    while True:
        found = set()
        for u in layer:
            looks += len(ends[u])
            found.update(v for i, v in ends[u] if x[i] and v not in placed)
        if not found:
            return False, built, looks
        placed |= found
        built += 1
        if t in found:
            return True, built, looks
        layer = found
