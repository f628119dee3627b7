"""Seeded generators for simple undirected typed graphs in CSR form.

Every generator returns a :class:`Graph`: ``row_ptr`` (int64, n+1),
``col`` (int32, 2M, each row sorted ascending, symmetric, no self-loops or
duplicates) and ``types`` (uint8, n, values in ``[0, L)``).

Seeds: ``numpy.random.default_rng`` (PCG64) seeded from a
``numpy.random.SeedSequence``; independent purposes (topology, types, ...)
draw from separate children of that sequence so one stream never shifts
another.

The workloads follow the shapes the paper evaluates on (Erdos-Renyi,
Chung-Lu power-law and k-partite heterogeneous graphs with types drawn at
random; Sec. 8, synthetic graph experiments) at the sizes the benchmark
configurations name.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class Graph:
    row_ptr: np.ndarray  # int64 [n+1]
    col: np.ndarray  # int32 [2M]
    types: np.ndarray  # uint8 [n]
    L: int
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    @property
    def m(self) -> int:
        return self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr)

    def edges(self) -> np.ndarray:
        """Undirected edges (u < v) in lexicographic order, int64 [M, 2]."""
        src = np.repeat(np.arange(self.n, dtype=np.int64), self.degrees())
        dst = self.col.astype(np.int64)
        keep = src < dst
        return np.stack([src[keep], dst[keep]], axis=1)

    def stats(self) -> dict:
        d = self.degrees().astype(np.float64)
        e = self.edges()
        same = 0.0
        if e.shape[0]:
            same = float(np.mean(self.types[e[:, 0]] == self.types[e[:, 1]]))
        return {
            "name": self.name,
            "n": self.n,
            "m": self.m,
            "L": self.L,
            "max_degree": int(d.max()) if d.size else 0,
            "sum_d2": float(np.sum(d * d)),
            "same_type_edge_fraction": same,
        }


def _rngs(seed, k):
    ss = np.random.SeedSequence(seed)
    return [np.random.default_rng(s) for s in ss.spawn(k)]


def csr_from_edges(n: int, u: np.ndarray, v: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Symmetric CSR of the simple graph spanned by pairs (u, v).

    Self-loops are dropped and duplicate pairs (in either direction) merged.
    Rows come out sorted ascending.
    """
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    keep = u != v
    u, v = u[keep], v[keep]
    lo = np.minimum(u, v)
    hi = np.maximum(u, v)
    key = np.unique(lo * n + hi)
    lo = key // n
    hi = key - lo * n
    src = np.concatenate([lo, hi])
    dst = np.concatenate([hi, lo])
    order = np.argsort(src * n + dst, kind="stable")
    src = src[order]
    dst = dst[order]
    counts = np.bincount(src, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return row_ptr, dst.astype(np.int32)


def _sample_types(rng, n, L, probs=None):
    if probs is None:
        return rng.integers(0, L, size=n, dtype=np.int64).astype(np.uint8)
    return rng.choice(L, size=n, p=np.asarray(probs) / np.sum(probs)).astype(np.uint8)


def zipf_probs(L: int, s: float) -> np.ndarray:
    p = (np.arange(1, L + 1, dtype=np.float64)) ** (-s)
    return p / p.sum()


def er_graph(n: int, avg_degree: float, L: int, seed: int = 0, name: str = "") -> Graph:
    """G(n, p) with p = avg_degree / (n - 1); every pair i < j independently."""
    r_top, r_typ = _rngs(seed, 2)
    p = avg_degree / (n - 1)
    iu, ju = np.triu_indices(n, k=1)
    pick = r_top.random(iu.shape[0]) < p
    row_ptr, col = csr_from_edges(n, iu[pick], ju[pick])
    types = _sample_types(r_typ, n, L)
    return Graph(row_ptr, col, types, L, name or f"er_n{n}_d{avg_degree}_L{L}")


def _power_weights(n: int, beta: float, mean: float, wmax: float) -> np.ndarray:
    """w_v proportional to (v + v0)^(-1/(beta-1)); v0 solved so that
    w_0 / mean(w) = wmax / mean, then scaled so mean(w) = mean."""
    a = 1.0 / (beta - 1.0)
    target = wmax / mean
    v = np.arange(n, dtype=np.float64)

    def ratio(v0):
        w = (v + v0) ** (-a)
        return w[0] / w.mean()

    lo, hi = 1e-9, float(n)
    for _ in range(200):
        mid = math.sqrt(lo * hi)
        if ratio(mid) > target:
            lo = mid
        else:
            hi = mid
    w = (v + math.sqrt(lo * hi)) ** (-a)
    return w * (mean / w.mean())


def _draw(rng, cdf, size):
    x = rng.random(size) * cdf[-1]
    return np.searchsorted(cdf, x, side="right").clip(0, cdf.shape[0] - 1)


def chung_lu_typed(
    n: int,
    avg_degree: float,
    beta: float,
    wmax: float,
    L: int,
    type_probs=None,
    homophily: float | None = None,
    oversample: float = 1.0,
    seed: int = 0,
    name: str = "",
) -> Graph:
    """Chung-Lu power-law graph with typed nodes and optional type homophily.

    Multigraph sampling: ``oversample * n * avg_degree / 2`` endpoint pairs are
    drawn, the first endpoint with probability proportional to its weight.
    With probability h the second endpoint is drawn proportional to weight
    among nodes of the first endpoint's type, otherwise among all nodes.
    h = (target - q) / (1 - q), q = sum_t (W_t / W)^2, so that the expected
    fraction of same-type pairs is the requested homophily while the
    expected degree of every node stays proportional to its weight.
    Self-loops and duplicates are then dropped.
    """
    r_w, r_typ, r_e = _rngs(seed, 3)
    del r_w
    w = _power_weights(n, beta, avg_degree, wmax)
    types = _sample_types(r_typ, n, L, type_probs)
    m_draw = int(round(oversample * n * avg_degree / 2))
    cdf = np.cumsum(w)
    u = _draw(r_e, cdf, m_draw)
    v = _draw(r_e, cdf, m_draw)
    if homophily is not None:
        wt = np.bincount(types, weights=w, minlength=L)
        q = float(np.sum((wt / wt.sum()) ** 2))
        h = max(0.0, (homophily - q) / (1.0 - q))
        same = r_e.random(m_draw) < h
        tu = types[u]
        for t in range(L):
            sel = np.nonzero(same & (tu == t))[0]
            if sel.size == 0:
                continue
            members = np.nonzero(types == t)[0]
            cdf_t = np.cumsum(w[members])
            v[sel] = members[_draw(r_e, cdf_t, sel.size)]
    row_ptr, col = csr_from_edges(n, u, v)
    return Graph(row_ptr, col, types, L, name or f"chung_lu_n{n}_b{beta}_L{L}")


def tripartite_graph(
    sizes=(1_000_000, 200_000, 50_000),
    m_target: int = 20_000_000,
    split=(0.5, 0.3, 0.2),
    beta: float = 2.3,
    wmax: float = 5e4,
    oversample: float = 1.0,
    seed: int = 0,
    name: str = "",
) -> Graph:
    """Three node classes A/B/C (types 0/1/2); edges only between classes.

    Pair split AB:AC:BC = ``split``.  A endpoints are uniform; B and C
    endpoints are drawn proportional to power-law weights (exponent
    ``beta``, largest expected degree ``wmax``).
    """
    nA, nB, nC = sizes
    n = nA + nB + nC
    r_e, = _rngs(seed, 1)
    mAB, mAC, mBC = (int(round(oversample * m_target * s)) for s in split)
    degB = (mAB + mBC) / nB
    degC = (mAC + mBC) / nC
    cB = np.cumsum(_power_weights(nB, beta, degB, wmax))
    cC = np.cumsum(_power_weights(nC, beta, degC, wmax))
    us, vs = [], []
    us.append(r_e.integers(0, nA, size=mAB))
    vs.append(nA + _draw(r_e, cB, mAB))
    us.append(r_e.integers(0, nA, size=mAC))
    vs.append(nA + nB + _draw(r_e, cC, mAC))
    us.append(nA + _draw(r_e, cB, mBC))
    vs.append(nA + nB + _draw(r_e, cC, mBC))
    row_ptr, col = csr_from_edges(n, np.concatenate(us), np.concatenate(vs))
    types = np.concatenate(
        [np.zeros(nA, np.uint8), np.ones(nB, np.uint8), np.full(nC, 2, np.uint8)]
    )
    return Graph(row_ptr, col, types, 3, name or "tripartite")


def random_small_graph(n: int, p: float, L: int, seed: int) -> Graph:
    """Tiny G(n, p) with uniform types, for brute-force checks."""
    r_top, r_typ = _rngs(seed, 2)
    iu, ju = np.triu_indices(n, k=1)
    pick = r_top.random(iu.shape[0]) < p
    row_ptr, col = csr_from_edges(n, iu[pick], ju[pick])
    return Graph(row_ptr, col, _sample_types(r_typ, n, L), L, f"gnp_n{n}_p{p}_s{seed}")


# ---------------------------------------------------------------------------
# The five benchmark configurations.

CONFIG_NAMES = {
    1: "er_n2000_d8_L3",
    2: "chung_lu_n1M_m10M_b2.1_L5_zipf1.2_h0.6",
    3: "tripartite_1M_200k_50k_m20M_b2.3_L3",
    4: "batch_100k_lognormal_chung_lu_L4to8",
    5: "serving_poisson2000_loguniform_m1e2_1e6_L6",
}

# Chung-Lu calibration for the power-law configuration: multigraph sampling
# merges repeated hub pairs, so the requested largest weight and the number
# of drawn pairs are set above the targets (Delta ~ 5e4, M ~ 1e7) such that
# the realised graph lands on them.
_CL2 = dict(n=1_000_000, avg_degree=20.0, beta=2.1, wmax=8.5e4, oversample=1.102,
            homophily=0.612)
_TRI3 = dict(wmax=5e4, oversample=1.03)


def config_graph(k: int, seed: int = 0, scale: float = 1.0) -> Graph:
    """Graph of configuration k (1, 2 or 3).

    ``scale`` < 1 shrinks configurations 2 and 3 (node and edge counts) while
    keeping their degree-distribution shape; it is used for tests that must
    stay small.
    """
    if k == 1:
        return er_graph(2000, 8.0, 3, seed=seed, name=CONFIG_NAMES[1])
    if k == 2:
        n = int(round(_CL2["n"] * scale))
        wmax = _CL2["wmax"] * math.sqrt(scale)
        return chung_lu_typed(
            n, _CL2["avg_degree"], _CL2["beta"], wmax, 5,
            type_probs=zipf_probs(5, 1.2), homophily=_CL2["homophily"],
            oversample=_CL2["oversample"], seed=seed,
            name=CONFIG_NAMES[2] if scale == 1.0 else f"{CONFIG_NAMES[2]}_x{scale}",
        )
    if k == 3:
        sizes = tuple(max(4, int(round(s * scale))) for s in (1_000_000, 200_000, 50_000))
        return tripartite_graph(
            sizes=sizes, m_target=int(round(20_000_000 * scale)),
            wmax=_TRI3["wmax"] * math.sqrt(scale), oversample=_TRI3["oversample"],
            seed=seed,
            name=CONFIG_NAMES[3] if scale == 1.0 else f"{CONFIG_NAMES[3]}_x{scale}",
        )
    raise ValueError(f"config {k} is not a single graph")


@dataclasses.dataclass
class GraphBatch:
    """Many typed graphs as one disjoint-union CSR.

    Graph g owns nodes [node_ptr[g], node_ptr[g+1]) and types in [0, L[g]);
    no edge joins two graphs.  ``union.L`` is max(L).
    """
    union: Graph
    node_ptr: np.ndarray  # int64 [G+1]
    L: np.ndarray         # int32 [G]

    @property
    def G(self) -> int:
        return int(self.L.shape[0])

    def edge_ptr(self) -> np.ndarray:
        """Edge id range of each graph in the union's canonical edge order."""
        d = self.union.degrees()
        src = np.repeat(np.arange(self.union.n, dtype=np.int64), d)
        upper = np.bincount(src[self.union.col > src], minlength=self.union.n)
        eoff = np.concatenate([[0], np.cumsum(upper)])
        return eoff[self.node_ptr]

    def graph(self, g: int) -> Graph:
        """Graph g on its own (node ids shifted to start at 0)."""
        a, b = int(self.node_ptr[g]), int(self.node_ptr[g + 1])
        rp = self.union.row_ptr[a:b + 1] - self.union.row_ptr[a]
        col = self.union.col[self.union.row_ptr[a]:self.union.row_ptr[b]] - a
        return Graph(rp.astype(np.int64), col.astype(np.int32), self.union.types[a:b].copy(),
                     int(self.L[g]), f"batch_g{g}")


def batch_graphs(num_graphs: int = 100_000, seed: int = 0, beta: float = 2.5) -> GraphBatch:
    """The batched configuration: many small typed Chung-Lu graphs.

    n_g = clip(round(exp(N(4, 1))), 10, 500); average degree dbar_g ~ U(4, 12);
    L_g ~ U{4..8}; types uniform in [0, L_g).  Inside each graph, Chung-Lu
    with weights proportional to (v+1)^(-1/(beta-1)) scaled to mean dbar_g
    and capped at 2 sqrt(n_g dbar_g); round(n_g dbar_g / 2) endpoint pairs
    drawn proportional to weight, self-loops and repeats dropped.  All graphs
    draw from one seeded stream, vectorised over graphs.
    """
    r_par, r_w, r_e, r_t = _rngs(seed, 4)
    del r_w
    n = np.clip(np.round(np.exp(r_par.normal(4.0, 1.0, size=num_graphs))), 10, 500).astype(np.int64)
    dbar = r_par.uniform(4.0, 12.0, size=num_graphs)
    L = r_par.integers(4, 9, size=num_graphs).astype(np.int32)
    node_ptr = np.concatenate([[0], np.cumsum(n)]).astype(np.int64)
    N = int(node_ptr[-1])
    gid = np.repeat(np.arange(num_graphs), n)
    local = np.arange(N, dtype=np.int64) - node_ptr[gid]
    a = 1.0 / (beta - 1.0)
    w = (local + 1.0) ** (-a)
    mean_w = np.add.reduceat(w, node_ptr[:-1]) / n
    w = w * (dbar / mean_w)[gid]
    wmax = 2.0 * np.sqrt(n * dbar)
    w = np.minimum(w, wmax[gid])
    cdf = np.cumsum(w)
    start = np.concatenate([[0.0], cdf[node_ptr[1:-1] - 1]])
    mass = cdf[node_ptr[1:] - 1] - start
    m_draw = np.round(n * dbar / 2).astype(np.int64)
    eg = np.repeat(np.arange(num_graphs), m_draw)
    def pick():
        x = start[eg] + r_e.random(eg.shape[0]) * mass[eg]
        v = np.searchsorted(cdf, x, side="right")
        return np.clip(v, node_ptr[eg], node_ptr[eg + 1] - 1)
    u = pick()
    v = pick()
    row_ptr, col = csr_from_edges(N, u, v)
    types = np.floor(r_t.random(N) * L[gid]).astype(np.uint8)
    union = Graph(row_ptr, col, types, int(L.max()), f"batch_{num_graphs}")
    return GraphBatch(union, node_ptr, L)


def serving_requests(num_requests: int, rate: float = 2000.0, seed: int = 0,
                     m_lo: float = 1e2, m_hi: float = 1e6, beta: float = 2.2, L: int = 6):
    """Poisson arrival times and per-request graph parameters.

    Returns a list of dicts ``{"arrival": seconds, "m": edges, "n": nodes,
    "seed": int}``; :func:`serving_graph` materialises one request's graph.
    """
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(1)[0])
    gaps = rng.exponential(1.0 / rate, size=num_requests)
    arrivals = np.cumsum(gaps)
    ms = np.exp(rng.uniform(math.log(m_lo), math.log(m_hi), size=num_requests))
    reqs = []
    for r in range(num_requests):
        m = int(round(ms[r]))
        reqs.append({"arrival": float(arrivals[r]), "m": m, "n": max(8, m // 5),
                     "seed": int(seed * 1_000_003 + r), "beta": beta, "L": L})
    return reqs


def serving_graph(req: dict) -> Graph:
    n = req["n"]
    dbar = 2.0 * req["m"] / n
    wmax = min(math.sqrt(n * dbar) * 2.0, n - 1.0)
    return chung_lu_typed(n, dbar, req["beta"], max(wmax, dbar * 1.01), req["L"],
                          type_probs=zipf_probs(req["L"], 1.2), seed=req["seed"],
                          name=f"req_{req['seed']}")


def orient(g: Graph, mutual: float = 0.2, seed: int = 0) -> np.ndarray:
    """Arc directions of a directed graph whose underlying undirected graph
    is ``g``: uint8 per CSR slot (u -> col[s]), bit 0 = the arc u -> col[s],
    bit 1 = the arc col[s] -> u.  Each edge is reciprocal with probability
    ``mutual``, else one arc of a fair coin's direction."""
    (rng,) = _rngs(seed, 1)
    e = g.edges()
    r = rng.random(e.shape[0])
    code = np.where(r < mutual, 3, np.where(r < mutual + (1 - mutual) / 2, 1, 2)).astype(np.uint8)
    src = np.repeat(np.arange(g.n, dtype=np.int64), g.degrees())
    dst = g.col.astype(np.int64)
    lo, hi = np.minimum(src, dst), np.maximum(src, dst)
    # edge id of each slot: rank of (lo, hi) among the edges (lexicographic)
    eid = np.searchsorted(e[:, 0] * g.n + e[:, 1], lo * g.n + hi)
    c = code[eid]
    swapped = ((c & 1) << 1) | ((c >> 1) & 1)
    return np.where(src < dst, c, swapped).astype(np.uint8)
