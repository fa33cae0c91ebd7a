"""Seeded synthetic SDP instances: graphs, cost matrices, constraint rows, test matrices.

This module builds problem *inputs* only: it never evaluates any step of the
solver.  Both the CPU oracle and the GPU library consume what it returns.

An SDP instance follows the primal form (P) of Sec. 2.1:
    maximise <C, X>  s.t.  <A_k, X> = b_k (k not in I),  <A_k, X> <= b_k (k in I),  X PSD,
with
  * C a symmetric sparse matrix stored as CSR with both triangles and the
    diagonal (rowptr int64 [n+1], col int32 [nnz], val float64 [nnz]);
  * A given by triplets (k, i, j, v) with i <= j meaning <A_k, X> = sum v * X_ij,
    so A_k = v E_ii for i == j and v (E_ij + E_ji)/2 for i < j;
  * b (float64 [m]), is_ineq (uint8 [m], 1 for rows in I);
  * trace = tr(X*) (or a bound), used by the problem scaling of App. E.

Workload families (Sec. 5.1 and App. E.1 MaxCut, App. E.3 correlation clustering):
  * MaxCut: C = L/4 with L the weighted graph Laplacian, A_i = E_ii, b = 1, I empty.
  * Correlation clustering: C = W (signed weights on the edges), rows X_ii = 1 and
    -X_ij <= 0 for every edge.
The paper's DIMACS10 graphs are not available; the random graphs below stand in
for their shape (sparse Laplacians with 7-9 nonzeros per row, Table 1).
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np


@dataclass
class SDPProblem:
    n: int
    rowptr: np.ndarray   # int64 [n+1]
    col: np.ndarray      # int32 [nnz]
    val: np.ndarray      # float64 [nnz]
    a_row: np.ndarray    # int32 [nt]
    a_i: np.ndarray      # int32 [nt]
    a_j: np.ndarray      # int32 [nt]
    a_v: np.ndarray      # float64 [nt]
    b: np.ndarray        # float64 [m]
    is_ineq: np.ndarray  # uint8 [m]
    trace: float
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.b.shape[0])

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])


# --------------------------------------------------------------------------
# graphs: edge lists with i < j, no duplicates, no self-loops
# --------------------------------------------------------------------------

def _canon(i, j):
    lo = np.minimum(i, j)
    hi = np.maximum(i, j)
    return lo, hi


def random_edges(n: int, m: int, rng: np.random.Generator):
    """m distinct edges drawn uniformly from all n(n-1)/2 pairs (the G(n, m) model)."""
    total = n * (n - 1) // 2
    if m > total:
        raise ValueError("more edges than pairs")
    keys = np.empty(0, dtype=np.int64)
    while keys.size < m:
        need = int((m - keys.size) * 1.1) + 16
        i = rng.integers(0, n, size=need, dtype=np.int64)
        j = rng.integers(0, n, size=need, dtype=np.int64)
        ok = i != j
        lo, hi = _canon(i[ok], j[ok])
        keys = np.unique(np.concatenate([keys, lo * n + hi]))
    if keys.size > m:
        keys = rng.permutation(keys)[:m]
        keys.sort()
    return (keys // n).astype(np.int64), (keys % n).astype(np.int64)


def erdos_renyi(n: int, p: float, rng: np.random.Generator):
    """G(n, p): every pair independently with probability p (edge count ~ Binomial)."""
    total = n * (n - 1) // 2
    m = int(rng.binomial(total, p))
    return random_edges(n, m, rng)


def random_regular(n: int, d: int, rng: np.random.Generator, bipartite: bool = False):
    """Random d-regular simple graph by the pairing (configuration) model with repair.

    bipartite=True gives a random d-regular bipartite graph between vertices
    [0, n/2) and [n/2, n) (n even), whose MaxCut value with unit weights is |E|.
    """
    if bipartite:
        if n % 2:
            raise ValueError("bipartite regular graph needs even n")
        h = n // 2
        left = np.repeat(np.arange(h, dtype=np.int64), d)
        right = rng.permutation(np.repeat(np.arange(h, n, dtype=np.int64), d))
        for _ in range(200):
            key = left * n + right
            order = np.argsort(key, kind="stable")
            dup = np.zeros(key.size, dtype=bool)
            dup[order[1:]] = key[order[1:]] == key[order[:-1]]
            bad = np.nonzero(dup)[0]
            if bad.size == 0:
                break
            # re-deal the right stubs of the bad pairs together with random others
            others = rng.choice(key.size, size=min(key.size, 4 * bad.size + 8), replace=False)
            sel = np.unique(np.concatenate([bad, others]))
            right[sel] = rng.permutation(right[sel])
        else:
            raise RuntimeError("pairing repair did not converge")
        lo, hi = _canon(left, right)
    else:
        if (n * d) % 2:
            raise ValueError("n*d must be even")
        stubs = rng.permutation(np.repeat(np.arange(n, dtype=np.int64), d))
        for _ in range(200):
            a, b = stubs[0::2], stubs[1::2]
            lo, hi = _canon(a, b)
            key = lo * n + hi
            order = np.argsort(key, kind="stable")
            dup = np.zeros(key.size, dtype=bool)
            dup[order[1:]] = key[order[1:]] == key[order[:-1]]
            bad = np.nonzero(dup | (lo == hi))[0]
            if bad.size == 0:
                break
            others = rng.choice(key.size, size=min(key.size, 4 * bad.size + 8), replace=False)
            sel = np.unique(np.concatenate([bad, others]))
            pos = np.concatenate([2 * sel, 2 * sel + 1])
            stubs[pos] = rng.permutation(stubs[pos])
        else:
            raise RuntimeError("pairing repair did not converge")
    order = np.lexsort((hi, lo))
    return lo[order], hi[order]


def complete_graph(n: int):
    i, j = np.triu_indices(n, 1)
    return i.astype(np.int64), j.astype(np.int64)


def cycle_graph(n: int):
    i = np.arange(n, dtype=np.int64)
    return _canon(i, (i + 1) % n)


def star_graph(n: int):
    j = np.arange(1, n, dtype=np.int64)
    return np.zeros(n - 1, dtype=np.int64), j


def hypercube_graph(d: int):
    n = 1 << d
    lo, hi = [], []
    for v in range(n):
        for b in range(d):
            u = v ^ (1 << b)
            if v < u:
                lo.append(v)
                hi.append(u)
    return np.array(lo, dtype=np.int64), np.array(hi, dtype=np.int64)


# --------------------------------------------------------------------------
# sparse symmetric matrices
# --------------------------------------------------------------------------

def sym_csr(n: int, i: np.ndarray, j: np.ndarray, w: np.ndarray, diag: np.ndarray | None):
    """CSR (both triangles + diagonal, columns sorted) of sum_e w_e (E_ij + E_ji) + Diag(diag)."""
    rows = [i, j]
    cols = [j, i]
    vals = [w, w]
    if diag is not None:
        rows.append(np.arange(n, dtype=np.int64))
        cols.append(np.arange(n, dtype=np.int64))
        vals.append(np.asarray(diag, dtype=np.float64))
    r = np.concatenate(rows).astype(np.int64)
    c = np.concatenate(cols).astype(np.int64)
    v = np.concatenate(vals).astype(np.float64)
    order = np.lexsort((c, r))
    r, c, v = r[order], c[order], v[order]
    # merge duplicates (none for simple graphs, kept for safety)
    key = r * n + c
    uniq, start = np.unique(key, return_index=True)
    if uniq.size != key.size:
        v = np.add.reduceat(v, start)
        r, c = uniq // n, uniq % n
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, r + 1, 1)
    rowptr = np.cumsum(rowptr)
    return rowptr, c.astype(np.int32), v


def laplacian_csr(n: int, i: np.ndarray, j: np.ndarray, w: np.ndarray, scale: float = 1.0):
    """CSR of scale * L with L = D - W the weighted Laplacian of the edge list."""
    deg = np.zeros(n, dtype=np.float64)
    np.add.at(deg, i, w)
    np.add.at(deg, j, w)
    return sym_csr(n, i, j, -scale * w, scale * deg)


# --------------------------------------------------------------------------
# problem families
# --------------------------------------------------------------------------

def maxcut_problem(n: int, i, j, w, name: str = "maxcut", meta: dict | None = None) -> SDPProblem:
    """MaxCut SDP of eq. maxcut_sdp: maximise (1/4) tr(L X) s.t. diag(X) = 1, X PSD."""
    i = np.asarray(i, dtype=np.int64)
    j = np.asarray(j, dtype=np.int64)
    w = np.asarray(w, dtype=np.float64)
    rowptr, col, val = laplacian_csr(n, i, j, w, 0.25)
    ar = np.arange(n, dtype=np.int32)
    md = {"edges_i": i, "edges_j": j, "weights": w}
    md.update(meta or {})
    return SDPProblem(
        n=n, rowptr=rowptr, col=col, val=val,
        a_row=ar.copy(), a_i=ar.copy(), a_j=ar.copy(), a_v=np.ones(n),
        b=np.ones(n), is_ineq=np.zeros(n, dtype=np.uint8), trace=float(n),
        name=name, meta=md)


def cc_problem(n: int, i, j, w, name: str = "cc", meta: dict | None = None) -> SDPProblem:
    """Correlation-clustering SDP (the core of eq. sdp_cc_w_econstraints on a sparse graph):
    maximise <W, X> s.t. X_vv = 1 for all v, X_ij >= 0 on every edge, X PSD.
    The inequality rows are written as <A_e, X> = -X_ij <= 0, i.e. triplet (e, i, j, -1), b_e = 0.
    """
    i = np.asarray(i, dtype=np.int64)
    j = np.asarray(j, dtype=np.int64)
    w = np.asarray(w, dtype=np.float64)
    rowptr, col, val = sym_csr(n, i, j, w, None)
    ne = i.size
    ar = np.arange(n, dtype=np.int32)
    er = (n + np.arange(ne)).astype(np.int32)
    md = {"edges_i": i, "edges_j": j, "weights": w}
    md.update(meta or {})
    return SDPProblem(
        n=n, rowptr=rowptr, col=col, val=val,
        a_row=np.concatenate([ar, er]),
        a_i=np.concatenate([ar, i.astype(np.int32)]),
        a_j=np.concatenate([ar, j.astype(np.int32)]),
        a_v=np.concatenate([np.ones(n), -np.ones(ne)]),
        b=np.concatenate([np.ones(n), np.zeros(ne)]),
        is_ineq=np.concatenate([np.zeros(n, dtype=np.uint8), np.ones(ne, dtype=np.uint8)]),
        trace=float(n), name=name, meta=md)


def test_matrix(n: int, r: int, seed: int) -> np.ndarray:
    """Gaussian test matrix Psi (n x r, i.i.d. N(0,1)) of the Nystrom sketch (Sec. 4),
    stored in float32; both solvers read exactly these values.  Row i depends only on
    (seed, i), so growing n keeps the old rows (warm starts)."""
    out = np.empty((n, r), dtype=np.float32)
    blk = 65536
    for s in range(0, n, blk):
        e = min(n, s + blk)
        rng = np.random.default_rng([seed, 0x5A17, s // blk])
        out[s:e] = rng.standard_normal((e - s, r)).astype(np.float32)
    return out


# --------------------------------------------------------------------------
# the workloads named for this method (synthetic stand-ins)
# --------------------------------------------------------------------------

def maxcut_er(n: int = 800, p: float = 0.02, seed: int = 0) -> SDPProblem:
    """Erdos-Renyi G(n, p), unit weights (default: n = 800, p = 0.02)."""
    rng = np.random.default_rng([seed, 1])
    i, j = erdos_renyi(n, p, rng)
    return maxcut_problem(n, i, j, np.ones(i.size), name=f"maxcut_er_n{n}_p{p}_s{seed}")


def maxcut_sparse_pm1(n: int = 20000, avg_degree: float = 6.0, seed: int = 0) -> SDPProblem:
    """n vertices, exactly n*deg/2 distinct uniform random edges, Rademacher +-1 weights."""
    rng = np.random.default_rng([seed, 2])
    m = int(round(n * avg_degree / 2))
    i, j = random_edges(n, m, rng)
    w = rng.choice(np.array([-1.0, 1.0]), size=m)
    return maxcut_problem(n, i, j, w, name=f"maxcut_pm1_n{n}_d{avg_degree}_s{seed}")


def maxcut_planted_pm1(n: int, avg_degree: float, seed: int = 0) -> SDPProblem:
    """Planted signed graph: hidden s in {+-1}^n, w_ij = +1 if s_i != s_j else -1.
    X = s s^T attains <L/4, X> = #positive edges, which also bounds every feasible X,
    so the SDP value is exactly the number of positive edges."""
    rng = np.random.default_rng([seed, 3])
    m = int(round(n * avg_degree / 2))
    i, j = random_edges(n, m, rng)
    s = rng.choice(np.array([-1.0, 1.0]), size=n)
    w = np.where(s[i] != s[j], 1.0, -1.0)
    return maxcut_problem(n, i, j, w, name=f"maxcut_planted_n{n}_s{seed}",
                          meta={"p_star": float(np.sum(w > 0)), "planted": s})


def maxcut_regular(n: int = 1_000_000, d: int = 4, seed: int = 0, bipartite: bool = False) -> SDPProblem:
    rng = np.random.default_rng([seed, 4])
    i, j = random_regular(n, d, rng, bipartite=bipartite)
    meta = {"p_star": float(i.size)} if bipartite else {}
    return maxcut_problem(n, i, j, np.ones(i.size),
                          name=f"maxcut_{'bip' if bipartite else ''}reg{d}_n{n}_s{seed}", meta=meta)


def cc_signed(n: int = 10000, avg_degree: float = 10.0, seed: int = 0, m_edges: int | None = None) -> SDPProblem:
    """Signed random graph with N(0,1) edge weights (correlation clustering)."""
    rng = np.random.default_rng([seed, 5])
    m = m_edges if m_edges is not None else int(round(n * avg_degree / 2))
    i, j = random_edges(n, m, rng)
    w = rng.standard_normal(m)
    return cc_problem(n, i, j, w, name=f"cc_n{n}_m{m}_s{seed}")


def served_batch(count: int = 256, n_lo: int = 500, n_hi: int = 5000, avg_degree: float = 8.0,
                 rate: float = 1.0, seed: int = 0):
    """Request trace of MaxCut SDPs: n ~ U{n_lo..n_hi}, G(n, deg/(n-1)), unit weights,
    Poisson arrivals of the given rate (requests per unit time).  Each entry also carries
    the grown instance (+ceil(1%) vertices, new edges with the same probability) used
    for the warm restart."""
    rng = np.random.default_rng([seed, 6])
    gaps = rng.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps) - gaps[0]
    reqs = []
    for r in range(count):
        n = int(rng.integers(n_lo, n_hi + 1))
        p = avg_degree / (n - 1)
        sub = np.random.default_rng([seed, 6, r])
        n2 = n + int(np.ceil(0.01 * n))
        i2, j2 = erdos_renyi(n2, p, sub)
        keep = (i2 < n) & (j2 < n)
        base = maxcut_problem(n, i2[keep], j2[keep], np.ones(int(keep.sum())), name=f"req{r}_n{n}")
        grown = maxcut_problem(n2, i2, j2, np.ones(i2.size), name=f"req{r}_n{n2}")
        reqs.append({"id": r, "arrival": float(t[r]), "problem": base, "grown": grown})
    return reqs


def general_overlap(n: int = 120, avg_degree: float = 6.0, n_rows: int = 40, terms: int = 3,
                    pool: int = 30, seed: int = 0) -> SDPProblem:
    """A general sparse constraint operator: C = W (signed graph, N(0,1) weights), rows
    X_vv = 1 for every v, then n_rows inequality rows  -sum_{(i,j) in S_k} X_ij <= 0.2  whose
    off-diagonal pairs S_k (terms each) are drawn from a small pool, so that the same pair
    appears in several rows (the form of the existence-constraint rows of Sec. 5.3)."""
    rng = np.random.default_rng([seed, 7])
    m_e = int(round(n * avg_degree / 2))
    i, j = random_edges(n, m_e, rng)
    w = rng.standard_normal(m_e)
    rowptr, col, val = sym_csr(n, i, j, w, None)
    pi, pj = random_edges(n, pool, rng)
    a_row = list(range(n))
    a_i = list(range(n))
    a_j = list(range(n))
    a_v = [1.0] * n
    for k in range(n_rows):
        pick = rng.choice(pool, size=terms, replace=False)
        for p in pick:
            a_row.append(n + k)
            a_i.append(int(pi[p]))
            a_j.append(int(pj[p]))
            a_v.append(-1.0)
    b = np.concatenate([np.ones(n), np.full(n_rows, 0.2)])
    ineq = np.concatenate([np.zeros(n, dtype=np.uint8), np.ones(n_rows, dtype=np.uint8)])
    return SDPProblem(
        n=n, rowptr=rowptr, col=col, val=val,
        a_row=np.asarray(a_row, dtype=np.int32), a_i=np.asarray(a_i, dtype=np.int32),
        a_j=np.asarray(a_j, dtype=np.int32), a_v=np.asarray(a_v, dtype=np.float64),
        b=b, is_ineq=ineq, trace=float(n), name=f"general_overlap_n{n}_s{seed}",
        meta={"edges_i": i, "edges_j": j, "weights": w})
