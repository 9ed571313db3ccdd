"""Seeded synthetic join graphs (query information) for the MPDP optimizer.

This module only draws inputs.  It holds none of the optimizer's arithmetic
(no cardinality estimation, no cost model, no enumeration), so both the CPU
oracle and the HIP path can consume the same arrays.

Query information follows the paper's QI (Section 2, Alg. 1 input): the
relations are vertices 0..n-1 of a join graph, each edge is an inner join
predicate.  Workload shapes follow the synthetic workloads of Section 7.2.1
(star, snowflake, clique) plus chains and cycles with extra chords.

Distributions (shared by every generator):
  * card[v] = 10 ** U(2, 8)                     (log-uniform 1e2 .. 1e8)
  * sel(u,v) = U(0.1, 1) / max(card[u], card[v]) (drawn in edge-list order)
All draws use ``numpy.random.Generator(PCG64(seed))``; topology first, then
cardinalities, then selectivities.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Query", "star", "snowflake", "chain", "cycle", "cycle_chords", "clique",
    "random_connected", "random_tree", "from_edges", "all_equal_clique", "batch_mixed", "large_snowflake",
]


@dataclass
class Query:
    """A join graph with statistics.

    n      number of relations (vertices 0..n-1)
    edges  (m, 2) uint32, one row per join predicate, u != v, no duplicates
    card   (n,) float64 base-relation cardinalities (finite, >= 1)
    sel    (m,) float64 selectivity of each edge, in (0, 1]
    name   free-form label of the workload and seed
    base_cost  optional (n,) float64: relation v is an intermediate result
           whose plan costs base_cost[v] (None: every relation is a scan)
    """
    n: int
    edges: np.ndarray
    card: np.ndarray
    sel: np.ndarray
    name: str = ""
    meta: dict = field(default_factory=dict)
    base_cost: np.ndarray | None = None

    @property
    def m(self) -> int:
        return int(self.edges.shape[0])

    def adjacency(self) -> list[int]:
        """Bitmap adjacency: bit u of adj[v] set iff (u, v) is an edge."""
        adj = [0] * self.n
        for u, v in self.edges.tolist():
            adj[u] |= 1 << v
            adj[v] |= 1 << u
        return adj


def _stats(rng: np.random.Generator, n: int, edges: np.ndarray):
    card = 10.0 ** rng.uniform(2.0, 8.0, size=n)
    if edges.shape[0]:
        mx = np.maximum(card[edges[:, 0]], card[edges[:, 1]])
        sel = rng.uniform(0.1, 1.0, size=edges.shape[0]) / mx
    else:
        sel = np.zeros(0, dtype=np.float64)
    return card.astype(np.float64), sel.astype(np.float64)


def from_edges(n: int, edges, seed: int, name: str = "") -> Query:
    """Query on a given topology with seeded statistics."""
    e = np.asarray(edges, dtype=np.uint32).reshape(-1, 2)
    rng = np.random.Generator(np.random.PCG64(seed))
    card, sel = _stats(rng, n, e)
    return Query(n, e, card, sel, name or f"custom{n}-s{seed}")


def star(n: int, seed: int) -> Query:
    """Hub 0 (fact relation) joined to leaves 1..n-1 (dimension relations)."""
    e = np.array([[0, i] for i in range(1, n)], dtype=np.uint32).reshape(-1, 2)
    rng = np.random.Generator(np.random.PCG64(seed))
    card, sel = _stats(rng, n, e)
    return Query(n, e, card, sel, f"star{n}-s{seed}")


def chain(n: int, seed: int) -> Query:
    e = np.array([[i, i + 1] for i in range(n - 1)], dtype=np.uint32).reshape(-1, 2)
    rng = np.random.Generator(np.random.PCG64(seed))
    card, sel = _stats(rng, n, e)
    return Query(n, e, card, sel, f"chain{n}-s{seed}")


def cycle(n: int, seed: int) -> Query:
    e = np.array([[i, (i + 1) % n] for i in range(n)], dtype=np.uint32).reshape(-1, 2)
    e = np.sort(e, axis=1)
    rng = np.random.Generator(np.random.PCG64(seed))
    card, sel = _stats(rng, n, e)
    return Query(n, e, card, sel, f"cycle{n}-s{seed}")


def clique(n: int, seed: int) -> Query:
    e = np.array([[i, j] for i in range(n) for j in range(i + 1, n)],
                 dtype=np.uint32).reshape(-1, 2)
    rng = np.random.Generator(np.random.PCG64(seed))
    card, sel = _stats(rng, n, e)
    return Query(n, e, card, sel, f"clique{n}-s{seed}")


def all_equal_clique(n: int, card: float = 1000.0, sel: float = 0.001) -> Query:
    """Clique with identical statistics everywhere: a storm of exact cost ties."""
    e = np.array([[i, j] for i in range(n) for j in range(i + 1, n)],
                 dtype=np.uint32).reshape(-1, 2)
    return Query(n, e, np.full(n, card), np.full(e.shape[0], sel), f"tieclique{n}")


def snowflake(n: int, seed: int, depth: int = 3, fanout=(2, 4)) -> Query:
    """Snowflake: root 0, breadth-first labelling, every node above ``depth``
    draws U{fanout} children; truncated at n nodes.  A tree that ends short of
    n nodes is redrawn from the same generator."""
    rng = np.random.Generator(np.random.PCG64(seed))
    while True:
        parent = [-1]
        lvl = [0]
        head = 0
        while head < len(parent) and len(parent) < n:
            if lvl[head] < depth:
                k = int(rng.integers(fanout[0], fanout[1] + 1))
                for _ in range(k):
                    if len(parent) >= n:
                        break
                    parent.append(head)
                    lvl.append(lvl[head] + 1)
            head += 1
        if len(parent) == n:
            break
    e = np.array([[parent[c], c] for c in range(1, n)], dtype=np.uint32).reshape(-1, 2)
    card, sel = _stats(rng, n, e)
    return Query(n, e, card, sel, f"snowflake{n}-s{seed}", {"depth": max(lvl)})


def cycle_chords(seed: int, n: int | None = None, chords: int | None = None,
                 n_range=(20, 30), chord_range=(5, 15)) -> Query:
    """Ring 0-1-..-(n-1)-0 plus distinct random chords, n ~ U{n_range} and
    chords ~ U{chord_range} unless given."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if n is None:
        n = int(rng.integers(n_range[0], n_range[1] + 1))
    if chords is None:
        chords = int(rng.integers(chord_range[0], chord_range[1] + 1))
    have = {(min(i, (i + 1) % n), max(i, (i + 1) % n)) for i in range(n)}
    cand = [(i, j) for i in range(n) for j in range(i + 1, n) if (i, j) not in have]
    pick = rng.choice(len(cand), size=min(chords, len(cand)), replace=False)
    es = sorted(have) + sorted(cand[int(p)] for p in pick)
    e = np.array(es, dtype=np.uint32).reshape(-1, 2)
    card, sel = _stats(rng, n, e)
    return Query(n, e, card, sel, f"cycle{n}+{chords}-s{seed}")


def random_tree(n: int, seed: int) -> Query:
    """Uniform random recursive tree with shuffled labels."""
    rng = np.random.Generator(np.random.PCG64(seed))
    perm = rng.permutation(n)
    es = []
    for i in range(1, n):
        j = int(rng.integers(0, i))
        a, b = int(perm[i]), int(perm[j])
        es.append((min(a, b), max(a, b)))
    e = np.array(es, dtype=np.uint32).reshape(-1, 2)
    card, sel = _stats(rng, n, e)
    return Query(n, e, card, sel, f"rtree{n}-s{seed}")


def random_connected(n: int, seed: int, extra: float = 0.3) -> Query:
    """Random spanning tree plus each remaining pair with probability ``extra``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    perm = rng.permutation(n)
    es = set()
    for i in range(1, n):
        j = int(rng.integers(0, i))
        a, b = int(perm[i]), int(perm[j])
        es.add((min(a, b), max(a, b)))
    for i in range(n):
        for j in range(i + 1, n):
            if (i, j) not in es and rng.random() < extra:
                es.add((i, j))
    e = np.array(sorted(es), dtype=np.uint32).reshape(-1, 2)
    card, sel = _stats(rng, n, e)
    return Query(n, e, card, sel, f"rconn{n}-p{extra}-s{seed}")


def batch_mixed(count: int, seed: int, n_range=(8, 20)) -> list[Query]:
    """Mixed batch: n ~ U{n_range}, topology uniform over chain, star, cycle
    (ring plus U{0..2} chords), snowflake (depth 3, fanout U{2..4}) and
    random (spanning tree plus U{1..3} extra edges); statistics as above.
    Query i uses the sub-seed (seed, i)."""
    kinds = ("chain", "star", "cycle", "snowflake", "random")
    out = []
    for i in range(count):
        rng = np.random.Generator(np.random.PCG64([seed, i]))
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        kind = kinds[int(rng.integers(0, len(kinds)))]
        s = int(rng.integers(0, 2 ** 31))
        if kind == "chain":
            q = chain(n, s)
        elif kind == "star":
            q = star(n, s)
        elif kind == "cycle" and n >= 3:
            q = cycle_chords(s, n=n, chords=int(rng.integers(0, 3)))
        elif kind == "cycle":
            q = chain(n, s)
        elif kind == "snowflake":
            q = snowflake(n, s)
        else:
            q = random_tree(n, s)
            extra = int(rng.integers(1, 4))
            have = {tuple(sorted(e)) for e in q.edges.tolist()}
            cand = [(a, b) for a in range(n) for b in range(a + 1, n) if (a, b) not in have]
            pick = rng.choice(len(cand), size=min(extra, len(cand)), replace=False)
            es = sorted(have) + sorted(cand[int(p)] for p in pick)
            q = from_edges(n, es, s, f"random{n}+{extra}-s{s}")
        q.name = f"batch{seed}/{i}:{q.name}"
        out.append(q)
    return out


def large_snowflake(n: int, seed: int, cross: int | None = None) -> Query:
    """Large snowflake with random cross edges (100-1000 relations): root 0,
    breadth-first labelling, every node above depth 4 draws U{2..F} children
    with F = max(4, ceil(2 n^(1/4))), truncated at n nodes (a tree that ends
    short is redrawn from the same generator); then ``cross`` (default
    round(n / 20)) distinct extra edges drawn uniformly among the non-edges."""
    rng = np.random.Generator(np.random.PCG64(seed))
    F = max(4, int(np.ceil(2.0 * n ** 0.25)))
    while True:
        parent, lvl, head = [-1], [0], 0
        while head < len(parent) and len(parent) < n:
            if lvl[head] < 4:
                for _ in range(int(rng.integers(2, F + 1))):
                    if len(parent) >= n:
                        break
                    parent.append(head)
                    lvl.append(lvl[head] + 1)
            head += 1
        if len(parent) == n:
            break
    es = {(parent[c], c) for c in range(1, n)}
    extra = int(round(n / 20)) if cross is None else int(cross)
    added = 0
    while added < extra:
        a, b = (int(x) for x in rng.integers(0, n, size=2))
        e = (min(a, b), max(a, b))
        if a == b or e in es:
            continue
        es.add(e)
        added += 1
    e = np.array(sorted(es), dtype=np.uint32).reshape(-1, 2)
    card, sel = _stats(rng, n, e)
    return Query(n, e, card, sel, f"lsnow{n}+{extra}-s{seed}", {"depth": max(lvl)})
