"""GPU parity at the full workload sizes, in the launch configuration the benchmark times.

The oracle cannot form these matrices densely; it checks what it can compute directly:
rows of the sparse operator product (scipy CSR, all rows), the low-rank constraint map on
every row, lambda_max by its Lanczos evaluator on the coupled rows plus the exact decoupled
diagonal, and the closed form p* = |E| of a bipartite 4-regular graph at n = 10^6.
"""
import numpy as np
import pytest

import sdp_inputs as si
from oracle import usbs_oracle as orc

pytestmark = pytest.mark.gpu

_CACHE = {}


def _problem(kind):
    if kind not in _CACHE:
        if kind == "c2":
            _CACHE[kind] = (si.maxcut_sparse_pm1(20000, 6.0, seed=0), "f32", 10, 1)
        elif kind == "c4":
            _CACHE[kind] = (si.cc_signed(10000, avg_degree=10.0, seed=0), "f32", 3, 0)
        else:
            _CACHE[kind] = (si.maxcut_regular(1_000_000, 4, seed=0, bipartite=True), "bf16", 10, 1)
    return _CACHE[kind]


def _dev(a, torch):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("kind,tol", [("c2", 2e-6), ("c4", 2e-6), ("c5", 2e-6)])
def test_fullsize_operator_rows(cuda, kind, tol):
    """Y = (C_s - A^* y) X for an 8-column block at full size against the oracle's sparse
    product, row by row.  c5's unit weights are exact in BF16 (one common scale), so the
    BF16 products only carry FP32 accumulation error; c4's y includes the edge rows, so the
    refreshed off-diagonal values are covered."""
    import torch
    from paper_2312_11801_amd import Params, Solver
    prob, prec, kc, kp = _problem(kind)
    rng = np.random.default_rng(5)
    sigma = float(np.linalg.norm(prob.val))
    y = rng.standard_normal(prob.m) * 0.5 / sigma
    X = rng.standard_normal((prob.n, 8))
    s = Solver(prob, Params(precision=prec, k_c=kc, k_p=kp, max_iters=1))
    Y = torch.zeros((prob.n, 8), dtype=torch.float64, device="cuda")
    s.op_apply(_dev(y, torch), _dev(X, torch), Y)
    torch.cuda.synchronize()
    got = Y.cpu().numpy()
    s.free()
    ref = orc.sparse_shifted(prob, y) @ X
    scale = np.abs(ref).max()
    err = np.abs(got - ref).max() / scale
    print(kind, "max rel err", err)
    assert err <= tol


def test_fullsize_lowrank_A_c4(cuda):
    """(A(W diag(lam) W^T))_k on all 60,000 rows (diagonal and edge rows) at n = 10,000."""
    import torch
    from paper_2312_11801_amd import Params, Solver
    prob, prec, kc, kp = _problem("c4")
    rng = np.random.default_rng(6)
    W = rng.standard_normal((prob.n, 3))
    lam = rng.random(3)
    s = Solver(prob, Params(precision=prec, k_c=kc, k_p=kp, max_iters=1))
    out = torch.zeros(prob.m, dtype=torch.float64, device="cuda")
    s.op_lowrank_A(_dev(W, torch), lam, out)
    got = out.cpu().numpy()
    s.free()
    ref = orc.A_lowrank(prob, W, lam)
    assert np.abs(got - ref).max() <= 1e-12 * (1 + np.abs(ref).max())


def test_fullsize_lambda_max_c2(cuda):
    """The eigen step's top Ritz value at n = 20,000 against the oracle's Lanczos on the
    coupled rows plus the exact diagonal of the decoupled rows: agreement within 1e-6
    relative to the spectral scale (FP32 operator values)."""
    import torch
    from paper_2312_11801_amd import Params, Solver
    prob, prec, kc, kp = _problem("c2")
    rng = np.random.default_rng(8)
    sigma = float(np.linalg.norm(prob.val))
    y = (1.0 + 0.2 * rng.standard_normal(prob.m)) * 1.2 / sigma
    s = Solver(prob, Params(precision=prec, k_c=kc, k_p=kp, max_iters=1, lanczos_tol=1e-9))
    w, res, cyc = s.op_eigs(_dev(y, torch), 4)
    s.free()
    ref = orc.lambda_max_sparse(prob, y, steps=400)
    M = orc.sparse_shifted(prob, y)
    scale = float(abs(M).sum(axis=1).max())
    print("gpu", w[0], "oracle", ref, "cycles", cyc)
    assert abs(w[0] - ref) <= 1e-6 * scale


def test_fullsize_c5_bipartite_closed_form(cuda):
    """n = 10^6 random bipartite 4-regular graph.  (1) With y_s = (d/2)/sigma on every vertex
    the shifted operator L/(4 sigma) - (d/2)/sigma I has lambda_max = 0 exactly (the top of
    L/4 is d/2 for a connected bipartite d-regular graph); the eigen step must return 0 to
    1e-6 of the spectral scale (the products accumulate in FP32, unit round-off 6e-8).  (2) A few iterations of the benchmark configuration end with
    a certified dual bound that satisfies weak duality against p* = |E| = 2n."""
    import torch
    from paper_2312_11801_amd import Params, Solver
    prob, prec, kc, kp = _problem("c5")
    p_star = prob.meta["p_star"]
    sigma = float(np.linalg.norm(prob.val))
    psi = si.test_matrix(prob.n, 10, seed=0)
    s = Solver(prob, Params(precision=prec, k_c=kc, k_p=kp, max_iters=5, lanczos_tol_final=1e-9), psi=psi)
    y = np.full(prob.m, 2.0 / sigma)
    w, res, cyc = s.op_eigs(_dev(y, torch), 2)
    print("lambda_max at the closed-form point", w[0], "cycles", cyc)
    assert abs(w[0]) <= 1e-6 * (4.0 / sigma)
    out = s.solve()
    s.free()
    print({k: out[k] for k in ("iters", "dual_bound", "primal_obj", "rel_gap", "seconds")}, "p*", p_star)
    assert out["dual_bound"] >= p_star * (1 - 1e-6)


@pytest.mark.parametrize("kind", ["c2", "c4"])
def test_fullsize_solve_certified(cuda, kind):
    """A cold solve at full size in the benchmark's configuration (restart cap 3 for the
    MaxCut graph, the paper's 10 for correlation clustering) reaches the 1e-3 criterion,
    and the oracle certifies it: f(y) from its Lanczos evaluator on the sparse matrix,
    A X_{t+1} and <C, X_{t+1}> rebuilt from the exported state, both relative errors
    (Sec. 5, eq. relative_error_tol), and the sketch's objective and infeasibility
    recomputed from its factors."""
    import sys
    from certify import certify
    from paper_2312_11801_amd import Params, Solver
    prob, prec, kc, kp = _problem(kind)
    psi = si.test_matrix(prob.n, 10, seed=0) if kind == "c2" else None
    maxr = 3 if kind == "c2" else 10
    s = Solver(prob, Params(precision=prec, k_c=kc, k_p=kp, max_iters=3000, lanczos_max_restarts=maxr), psi=psi)
    out = s.solve()
    print(kind, {k: out[k] for k in ("iters", "seconds", "rel_gap", "rel_infeas", "primal_obj", "dual_bound")},
          flush=True)
    assert out["converged"], out
    # the oracle's Lanczos is a lower bound of lambda_max like the library's Ritz value
    certify(prob, s, out, dense=False, f_tol=1e-6, say=lambda *a: print(*a, file=sys.stdout, flush=True))
    s.free()


def test_fullsize_c5_solve_certified(cuda):
    """The benchmark's headline configuration: n = 10^6 random 4-regular graph (not
    bipartite), FP64 products, restart cap 3, sketch rank 10, X never formed.  A cold solve
    reaches the 1e-3 criterion (scaled units, App. E) and the oracle certifies it: f(y) from
    120 steps of its Lanczos evaluator (a lower bound of lambda_max like the library's Ritz
    value; 60 more steps move it by about 2e-6 in f here, so f agrees to 1e-5 absolute),
    A X_{t+1} and <C, X_{t+1}> rebuilt from the exported state, both relative errors, and
    <C, Xhat> and A(Xhat) of the Nystrom reconstruction recomputed from its factors."""
    import sys
    from certify import certify
    from paper_2312_11801_amd import Params, Solver
    prob = si.maxcut_regular(1_000_000, 4, seed=0)
    psi = si.test_matrix(prob.n, 10, seed=0)
    s = Solver(prob, Params(precision="f64", max_iters=500, lanczos_max_restarts=3), psi=psi)
    out = s.solve()
    print({k: out[k] for k in ("iters", "seconds", "rel_gap", "rel_infeas", "primal_obj", "dual_bound",
                               "sketch_primal_obj", "sketch_rel_infeas")}, flush=True)
    assert out["converged"], out
    certify(prob, s, out, dense=False, f_tol=1e-5, lanczos_steps=120,
            say=lambda *a: print(*a, file=sys.stdout, flush=True))
    s.free()
