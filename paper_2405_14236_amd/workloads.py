"""Seeded synthetic inputs for the condensed-KKT solves.

This module only *draws* problem data (sparsity patterns, matrix values,
diagonals and right-hand sides).  It contains none of the method's
arithmetic: no condensation, no factorization, no residuals.  Both the CPU
oracle (through the tests) and the HIP path consume what it returns.

Shapes follow the paper's nonlinear program (Sec. 2.1, eq:slack_problem):
``n`` primal variables, ``m_eq`` equality rows with Jacobian G and ``m_ineq``
inequality rows with Jacobian H.  The Hessian W is given by its lower
triangle.  The diagonals are

* ``sigma_x`` (length n): the primal diagonal (delta_w I of K2, generalised to
  any nonnegative diagonal),
* ``sigma_s`` (length m_eq + m_ineq): the per-row diagonal D_H of the
  condensed matrix (Sec. 2.2, K1).  LiftedKKT uses all of it (equalities are
  relaxed into tight inequality rows, Sec. 3.2, eq:liftedkkt); HyKKT uses
  the inequality part ``sigma_s[m_eq:]`` and weighs G by gamma
  (Sec. 3.1, eq:kkt:hykkt).

All matrices are CSR with int32 indices (sorted, no duplicates) and float64
values.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np


@dataclasses.dataclass
class KKTProblem:
    n: int
    m_eq: int
    m_ineq: int
    w_ptr: np.ndarray
    w_idx: np.ndarray
    w_val: np.ndarray
    g_ptr: np.ndarray
    g_idx: np.ndarray
    g_val: np.ndarray
    h_ptr: np.ndarray
    h_idx: np.ndarray
    h_val: np.ndarray
    sigma_x: np.ndarray
    sigma_s: np.ndarray
    b: np.ndarray          # LiftedKKT right-hand side (length n)
    r1bar: np.ndarray      # HyKKT / K1 first block (length n)
    r2bar: np.ndarray      # HyKKT / K1 second block (length m_eq)
    gamma: float = 1e7
    name: str = ""

    @property
    def m(self) -> int:
        return self.m_eq + self.m_ineq

    @property
    def sigma_s_ineq(self) -> np.ndarray:
        return self.sigma_s[self.m_eq:]

    def with_sigma(self, sigma_x: np.ndarray, sigma_s: np.ndarray) -> "KKTProblem":
        return dataclasses.replace(self, sigma_x=np.ascontiguousarray(sigma_x, dtype=np.float64),
                                   sigma_s=np.ascontiguousarray(sigma_s, dtype=np.float64))


# --------------------------------------------------------------------------
# small helpers (pattern bookkeeping only)
# --------------------------------------------------------------------------

def _csr_from_rows(rows: List[dict], ncols: int):
    """rows[i] maps column -> value.  Returns sorted CSR arrays."""
    ptr = np.zeros(len(rows) + 1, dtype=np.int32)
    for i, r in enumerate(rows):
        ptr[i + 1] = ptr[i] + len(r)
    idx = np.empty(int(ptr[-1]), dtype=np.int32)
    val = np.empty(int(ptr[-1]), dtype=np.float64)
    for i, r in enumerate(rows):
        cols = sorted(r)
        a = int(ptr[i])
        idx[a:a + len(cols)] = cols
        val[a:a + len(cols)] = [r[c] for c in cols]
    assert (idx >= 0).all() and (idx < max(ncols, 1)).all() if len(idx) else True
    return ptr, idx, val


def _csr_from_coo(nrows: int, rows: np.ndarray, cols: np.ndarray, vals: np.ndarray):
    """Sorted CSR from COO triplets that hold no duplicate positions."""
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    if len(rows) > 1:
        dup = (rows[1:] == rows[:-1]) & (cols[1:] == cols[:-1])
        assert not dup.any(), "duplicate entries in generator"
    ptr = np.zeros(nrows + 1, dtype=np.int64)
    np.add.at(ptr, rows + 1, 1)
    ptr = np.cumsum(ptr).astype(np.int32)
    return ptr, cols.astype(np.int32), vals.astype(np.float64)


def log_uniform(rng: np.random.Generator, size, lo_exp=-8.0, hi_exp=8.0) -> np.ndarray:
    return 10.0 ** rng.uniform(lo_exp, hi_exp, size=size)


def lattice_edges(N: int):
    """Edges of a row-major lattice holding nodes 0..N-1, ceil(sqrt N) columns."""
    sx = int(math.ceil(math.sqrt(N)))
    k = np.arange(N)
    horiz = k[(k % sx != sx - 1) & (k + 1 < N)]
    vert = k[k + sx < N]
    e = np.concatenate([np.stack([horiz, horiz + 1], 1), np.stack([vert, vert + sx], 1)])
    return e.astype(np.int64)


def _random_spanning_tree(rng, N, cand):
    """Kruskal on random weights: a random spanning tree of the candidate graph."""
    parent = np.arange(N)

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    order = rng.permutation(len(cand))
    in_tree = np.zeros(len(cand), dtype=bool)
    cnt = 0
    for t in order:
        a, b = cand[t]
        ra, rb = find(a), find(b)
        if ra != rb:
            parent[ra] = rb
            in_tree[t] = True
            cnt += 1
            if cnt == N - 1:
                break
    assert cnt == N - 1, "candidate graph is not connected"
    return in_tree


def network_graph(rng, N: int, E: int, topology: str = "grid") -> np.ndarray:
    """Random connected sparse graph with N nodes and E edges.

    ``grid``: a random spanning tree of a lattice plus extra lattice edges
    (planar, power-network-like).  ``uniform``: a random tree plus uniform
    random chords (an expander, much more fill).
    """
    if topology == "grid":
        cand = lattice_edges(N)
        if E > len(cand):
            raise ValueError("too many edges for the lattice")
        in_tree = _random_spanning_tree(rng, N, cand)
        rest = np.flatnonzero(~in_tree)
        extra = rng.choice(rest, size=E - (N - 1), replace=False)
        edges = np.concatenate([cand[in_tree], cand[extra]])
    elif topology == "uniform":
        # random recursive tree + uniform chords
        tree = [(int(rng.integers(0, i)), i) for i in range(1, N)]
        have = set(tree)
        edges = list(tree)
        while len(edges) < E:
            a, b = sorted(int(v) for v in rng.integers(0, N, size=2))
            if a != b and (a, b) not in have:
                have.add((a, b))
                edges.append((a, b))
        edges = np.array(edges, dtype=np.int64)
    else:
        raise ValueError(topology)
    return edges[rng.permutation(len(edges))]


def _spd_block(rng, k):
    B = rng.standard_normal((k, k))
    return B @ B.T + 0.1 * np.eye(k)


# --------------------------------------------------------------------------
# workload 1: tiny 2-D grid problem (n = 300)
# --------------------------------------------------------------------------

def tiny_grid(seed: int = 0, nx: int = 10, ny: int = 10, vpn: int = 3,
              m_eq: Optional[int] = None, m_ineq: Optional[int] = None,
              sigma_range=(-8.0, 8.0)) -> KKTProblem:
    """Grid graph of nx*ny nodes, ``vpn`` variables per node.

    W: dense vpn x vpn block inside each node plus two random couplings per
    grid edge, N(0,1) values, then a Gershgorin diagonal shift so that W is
    SPD (hence positive definite on Ker(J)).
    J: about four nonzeros per row among a node's and its neighbours'
    variables; row r of G always holds the node variable ``vpn*u + r // N``
    so that G has a structurally full row rank.
    """
    rng = np.random.default_rng(seed)
    N = nx * ny
    n = vpn * N
    if m_eq is None:
        m_eq = (2 * n) // 5
    if m_ineq is None:
        m_ineq = n - m_eq
    nbrs = [[] for _ in range(N)]
    edges = []
    for y in range(ny):
        for x in range(nx):
            u = y * nx + x
            if x + 1 < nx:
                edges.append((u, u + 1))
            if y + 1 < ny:
                edges.append((u, u + nx))
    for a, b in edges:
        nbrs[a].append(b)
        nbrs[b].append(a)
    # W lower triangle
    Wd = [dict() for _ in range(n)]

    def addw(i, j, v):
        if i < j:
            i, j = j, i
        Wd[i][j] = Wd[i].get(j, 0.0) + v

    for u in range(N):
        for a in range(vpn):
            for c in range(a):
                addw(vpn * u + a, vpn * u + c, rng.standard_normal())
    for (u, v) in edges:
        for _ in range(2):
            a, c = rng.integers(0, vpn, size=2)
            addw(vpn * u + int(a), vpn * v + int(c), rng.standard_normal())
    offsum = np.zeros(n)
    for i in range(n):
        for j, v in Wd[i].items():
            offsum[i] += abs(v)
            offsum[j] += abs(v)
    for i in range(n):
        Wd[i][i] = offsum[i] + 1.0 + abs(rng.standard_normal())
    w_ptr, w_idx, w_val = _csr_from_rows(Wd, n)

    def jrow(u, forced=None):
        pool = [vpn * u + a for a in range(vpn)]
        for v in nbrs[u]:
            pool += [vpn * v + a for a in range(vpn)]
        cols = set(int(c) for c in rng.choice(pool, size=min(4, len(pool)), replace=False))
        if forced is not None:
            cols.add(forced)
        return {c: rng.standard_normal() for c in cols}

    G_rows = []
    for r in range(m_eq):
        u = r % N
        G_rows.append(jrow(u, forced=vpn * u + (r // N) % vpn))
    H_rows = [jrow((m_eq + r) % N) for r in range(m_ineq)]
    g_ptr, g_idx, g_val = _csr_from_rows(G_rows, n)
    h_ptr, h_idx, h_val = _csr_from_rows(H_rows, n)
    lo, hi = sigma_range
    sigma_x = log_uniform(rng, n, lo, hi)
    sigma_s = log_uniform(rng, m_eq + m_ineq, lo, hi)
    b = rng.standard_normal(n)
    r1 = rng.standard_normal(n)
    r2 = rng.standard_normal(m_eq)
    return KKTProblem(n, m_eq, m_ineq, w_ptr, w_idx, w_val, g_ptr, g_idx, g_val,
                      h_ptr, h_idx, h_val, sigma_x, sigma_s, b, r1, r2,
                      name=f"tiny_grid(seed={seed},n={n})")


# --------------------------------------------------------------------------
# workloads 2-4: network-flow-shaped NLP
# --------------------------------------------------------------------------

def network_flow(N: int = 10_000, E: Optional[int] = None, seed: int = 0,
                 topology: str = "grid", sigma_range=(-8.0, 8.0)) -> KKTProblem:
    """Network-flow-shaped problem on a random connected graph.

    * 4 variables per node, 2 per edge: n = 4N + 2E.
    * 2 equality rows per node: row (i, k) holds node i's 4 variables and
      variable k of every incident edge.
    * 4 inequality rows per edge (a, b): {e0}, {e1}, {e0, e1},
      {a_1, b_1, e0, e1}.
    * W: a 4x4 SPD block per node and a 2x2 SPD block per edge (B B^T + 0.1 I).
    * Jacobian values N(0,1); diagonals log-uniform in 10^[lo, hi].
    """
    rng = np.random.default_rng(seed)
    if E is None:
        E = int(round(1.3 * N))
    edges = network_graph(rng, N, E, topology)
    n = 4 * N + 2 * E
    m_eq = 2 * N
    m_ineq = 4 * E
    ev = 4 * N + 2 * np.arange(E)  # first variable of each edge

    # W: node blocks and edge blocks, lower triangles
    wr, wc, wv = [], [], []
    nb = rng.standard_normal((N, 4, 4))
    nodeblk = nb @ nb.transpose(0, 2, 1) + 0.1 * np.eye(4)
    eb = rng.standard_normal((E, 2, 2))
    edgeblk = eb @ eb.transpose(0, 2, 1) + 0.1 * np.eye(2)
    base = 4 * np.arange(N)
    for a in range(4):
        for c in range(a + 1):
            wr.append(base + a); wc.append(base + c); wv.append(nodeblk[:, a, c])
    for a in range(2):
        for c in range(a + 1):
            wr.append(ev + a); wc.append(ev + c); wv.append(edgeblk[:, a, c])
    w_ptr, w_idx, w_val = _csr_from_coo(n, np.concatenate(wr), np.concatenate(wc),
                                        np.concatenate(wv))

    # G: node balance rows
    inc_node = np.concatenate([edges[:, 0], edges[:, 1]])
    inc_edge = np.concatenate([np.arange(E), np.arange(E)])
    gr, gc = [], []
    for k in range(2):
        rows_nodes = 2 * np.arange(N) + k
        for a in range(4):
            gr.append(rows_nodes); gc.append(base + a)
        gr.append(2 * inc_node + k); gc.append(ev[inc_edge] + k)
    gr = np.concatenate(gr); gc = np.concatenate(gc)
    # parallel edges cannot occur (simple graph), self loops neither
    g_ptr, g_idx, g_val = _csr_from_coo(m_eq, gr, gc, rng.standard_normal(len(gr)))

    # H: four rows per edge
    e = np.arange(E)
    a_n, b_n = edges[:, 0], edges[:, 1]
    hr = [4 * e, 4 * e + 1, 4 * e + 2, 4 * e + 2,
          4 * e + 3, 4 * e + 3, 4 * e + 3, 4 * e + 3]
    hc = [ev, ev + 1, ev, ev + 1, 4 * a_n + 1, 4 * b_n + 1, ev, ev + 1]
    hr = np.concatenate(hr); hc = np.concatenate(hc)
    h_ptr, h_idx, h_val = _csr_from_coo(m_ineq, hr, hc, rng.standard_normal(len(hr)))

    lo, hi = sigma_range
    sigma_x = log_uniform(rng, n, lo, hi)
    sigma_s = log_uniform(rng, m_eq + m_ineq, lo, hi)
    b = rng.standard_normal(n)
    r1 = rng.standard_normal(n)
    r2 = rng.standard_normal(m_eq)
    return KKTProblem(n, m_eq, m_ineq, w_ptr, w_idx, w_val, g_ptr, g_idx, g_val,
                      h_ptr, h_idx, h_val, sigma_x, sigma_s, b, r1, r2,
                      name=f"network_flow(N={N},E={E},{topology},seed={seed})")


def ipm_sigma_sequence(prob: KKTProblem, num: int, seed: int = 0,
                       active_frac: float = 0.3, exp: float = 8.0):
    """IPM-like diagonal sequence (centrality model of Prop. prop:cond:boundslack).

    Every diagonal entry j gets a target exponent e_j in {+exp, -exp}:
    relaxed-equality rows and a fraction ``active_frac`` of the inequality
    rows are active (D grows to 10^exp), the other rows and all primal
    entries shrink to 10^-exp.  Entry j of system k is 10^(e_j k / (num-1)),
    so system 0 is all ones.  Returns a list of (sigma_x, sigma_s).
    """
    rng = np.random.default_rng(seed + 7919)
    ex = -exp * np.ones(prob.n)
    es = np.empty(prob.m)
    es[:prob.m_eq] = exp
    act = rng.random(prob.m_ineq) < active_frac
    es[prob.m_eq:] = np.where(act, exp, -exp)
    out = []
    for k in range(num):
        t = k / max(num - 1, 1)
        out.append((10.0 ** (ex * t), 10.0 ** (es * t)))
    return out


def with_dense_rows(prob: KKTProblem, count: int = 4, frac: float = 0.5, seed: int = 0,
                    sigma_exp=(-8.0, 8.0), equality: bool = False) -> KKTProblem:
    """``prob`` with ``count`` extra rows, each over a random fraction ``frac``
    of the variables with N(0, 1) coefficients (budget- or resource-style
    constraints: the dense rows that fill the condensed matrix, Sec. 1 and
    Sec. 2.2).  Inequality rows (appended to H) get sigma_s entries drawn
    log-uniform like the others; equality rows (``equality``, appended to G)
    get sigma_s entries too (LiftedKKT relaxes them) and N(0, 1) entries of
    rbar2."""
    rng = np.random.default_rng(seed + 104_729)
    n = prob.n
    k = max(1, int(round(frac * n)))
    src_ptr, src_idx, src_val = ((prob.g_ptr, prob.g_idx, prob.g_val) if equality
                                 else (prob.h_ptr, prob.h_idx, prob.h_val))
    ptr = [int(x) for x in src_ptr]
    idx, val = list(src_idx), list(src_val)
    for _ in range(count):
        cols = np.sort(rng.choice(n, size=k, replace=False))
        idx.extend(int(c) for c in cols)
        val.extend(rng.standard_normal(k))
        ptr.append(len(idx))
    extra = log_uniform(rng, count, *sigma_exp)
    arrays = (np.asarray(ptr, dtype=np.int32), np.asarray(idx, dtype=np.int32), np.asarray(val, dtype=np.float64))
    name = f"{prob.name}+{count}dense{'eq' if equality else ''}{frac:g}"
    if equality:
        return dataclasses.replace(
            prob, m_eq=prob.m_eq + count, g_ptr=arrays[0], g_idx=arrays[1], g_val=arrays[2],
            sigma_s=np.concatenate([prob.sigma_s[:prob.m_eq], extra, prob.sigma_s[prob.m_eq:]]),
            r2bar=np.concatenate([prob.r2bar, rng.standard_normal(count)]), name=name)
    return dataclasses.replace(
        prob, m_ineq=prob.m_ineq + count, h_ptr=arrays[0], h_idx=arrays[1], h_val=arrays[2],
        sigma_s=np.concatenate([prob.sigma_s, extra]), name=name)


def batch_network_flow(count: int = 512, seed: int = 0, nmin: int = 500,
                       nmax: int = 2000) -> List[KKTProblem]:
    """Independent network-flow instances of uneven size (node counts U{nmin..nmax})."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(nmin, nmax + 1, size=count)
    return [network_flow(int(N), seed=seed * 100_003 + i + 1) for i, N in enumerate(sizes)]


# --------------------------------------------------------------------------
# workload 5: PDE-constrained-shaped NLP (3-D Laplacian)
# --------------------------------------------------------------------------

def pde_control(side: int = 48, alpha: float = 1e-2, seed: int = 0,
                sigma_range=(-8.0, 8.0)) -> KKTProblem:
    """Distributed control of a 3-D Poisson equation.

    States on a side^3 grid, controls on the stride-2 subgrid.  W is the
    7-point Dirichlet Laplacian on the states plus alpha*I on the controls;
    G = [L7 | -B] (one row per state, B injects each control at its grid
    point); H holds one bound row per control.
    """
    rng = np.random.default_rng(seed)
    ns = side ** 3
    cs = (side + 1) // 2
    nc = cs ** 3
    n = ns + nc
    idx3 = np.arange(ns).reshape(side, side, side)
    lr, lc, lv = [idx3.ravel()], [idx3.ravel()], [np.full(ns, 6.0)]
    for ax in range(3):
        a = np.take(idx3, np.arange(side - 1), axis=ax).ravel()
        b = np.take(idx3, np.arange(1, side), axis=ax).ravel()
        lr += [a, b]; lc += [b, a]; lv += [np.full(a.size, -1.0)] * 2
    lr = np.concatenate(lr); lc = np.concatenate(lc); lv = np.concatenate(lv)
    low = lr >= lc
    w_r = np.concatenate([lr[low], ns + np.arange(nc)])
    w_c = np.concatenate([lc[low], ns + np.arange(nc)])
    w_v = np.concatenate([lv[low], np.full(nc, alpha)])
    w_ptr, w_idx, w_val = _csr_from_coo(n, w_r, w_c, w_v)
    sub = idx3[::2, ::2, ::2].ravel()
    g_r = np.concatenate([lr, sub])
    g_c = np.concatenate([lc, ns + np.arange(nc)])
    g_v = np.concatenate([lv, -np.ones(nc)])
    g_ptr, g_idx, g_val = _csr_from_coo(ns, g_r, g_c, g_v)
    h_ptr = np.arange(nc + 1, dtype=np.int32)
    h_idx = (ns + np.arange(nc)).astype(np.int32)
    h_val = np.ones(nc)
    lo, hi = sigma_range
    sigma_x = log_uniform(rng, n, lo, hi)
    sigma_s = log_uniform(rng, ns + nc, lo, hi)
    b = rng.standard_normal(n)
    r1 = rng.standard_normal(n)
    r2 = rng.standard_normal(ns)
    return KKTProblem(n, ns, nc, w_ptr, w_idx, w_val, g_ptr, g_idx, g_val,
                      h_ptr, h_idx, h_val, sigma_x, sigma_s, b, r1, r2,
                      name=f"pde_control(side={side})")


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------

WORKLOADS = {
    "tiny_grid_n300": lambda seed=0: tiny_grid(seed),
    "netflow_N10k": lambda seed=0: network_flow(10_000, seed=seed),
    "netflow_N80k": lambda seed=0: network_flow(80_000, seed=seed),
    "pde_48": lambda seed=0: pde_control(48, seed=seed),
}


def workload(name: str, seed: int = 0) -> KKTProblem:
    return WORKLOADS[name](seed)
