"""Pins of the CPU oracle against facts the paper and the mathematics fix (no GPU).

Each test would fail for a plausible mistake in the oracle: a dropped term, a wrong
sign or index, a transposed operand, a wrong scaling.
"""
import math

import numpy as np
import pytest

import sdp_inputs as si
from oracle import usbs_oracle as orc


# ---------------------------------------------------------------------------
# Jacobi eigendecomposition vs closed-form Laplacian spectra
# ---------------------------------------------------------------------------
def _lap(n, i, j):
    L = np.zeros((n, n))
    for a, b in zip(i, j):
        L[a, b] -= 1
        L[b, a] -= 1
        L[a, a] += 1
        L[b, b] += 1
    return L


@pytest.mark.parametrize("n", [7, 16])
def test_jacobi_complete_graph(n):
    w, V = orc.jacobi_eigh(_lap(n, *si.complete_graph(n)))
    assert np.allclose(w[:-1], n, atol=1e-12) and abs(w[-1]) < 1e-12
    assert np.abs(V.T @ V - np.eye(n)).max() < 1e-13


def test_jacobi_cycle_star_hypercube():
    n = 13
    w = orc.jacobi_eigh(_lap(n, *si.cycle_graph(n)))[0]
    ref = np.sort(2 - 2 * np.cos(2 * np.pi * np.arange(n) / n))[::-1]
    assert np.abs(w - ref).max() < 1e-12
    w = orc.jacobi_eigh(_lap(9, *si.star_graph(9)))[0]
    assert np.abs(w - np.array([9] + [1] * 7 + [0])).max() < 1e-12
    d = 5
    w = orc.jacobi_eigh(_lap(1 << d, *si.hypercube_graph(d)))[0]
    ref = np.sort(np.concatenate([[2 * i] * math.comb(d, i) for i in range(d + 1)]))[::-1]
    assert np.abs(w - ref).max() < 1e-12


def test_jacobi_random_residual_and_order():
    rng = np.random.default_rng(0)
    A = rng.standard_normal((40, 40))
    A = A + A.T
    w, V = orc.jacobi_eigh(A)
    assert np.all(np.diff(w) <= 0)
    assert np.abs(A @ V - V * w).max() < 1e-12 * np.abs(w).max()
    assert np.abs(V.T @ V - np.eye(40)).max() < 1e-13
    assert abs(w.sum() - np.trace(A)) < 1e-11


# ---------------------------------------------------------------------------
# svec, U, symmetric Kronecker product (App. B)
# ---------------------------------------------------------------------------
def test_svec_inner_product_and_U():
    rng = np.random.default_rng(1)
    k = 5
    A = rng.standard_normal((k, k)); A = A + A.T
    B = rng.standard_normal((k, k)); B = B + B.T
    assert abs(orc.svec(A) @ orc.svec(B) - np.trace(A @ B)) < 1e-12
    U = orc.svec_U(k)
    vec = A.flatten(order="F")
    assert np.abs(U @ vec - orc.svec(A)).max() < 1e-13
    assert np.abs(U.T @ U @ vec - vec).max() < 1e-13
    assert np.abs(U @ U.T - np.eye(k * (k + 1) // 2)).max() < 1e-14   # orthonormal rows
    assert np.abs(orc.smat(orc.svec(A), k) - A).max() < 1e-14
    # the printed n = 2 example
    r = 1 / math.sqrt(2)
    assert np.allclose(orc.svec_U(2), [[1, 0, 0, 0], [0, r, r, 0], [0, 0, 0, 1]])


def test_skron_action():
    rng = np.random.default_rng(2)
    k = 4
    G = rng.standard_normal((k, k)); G = G + G.T
    H = rng.standard_normal((k, k)); H = H + H.T
    A = rng.standard_normal((k, k)); A = A + A.T
    lhs = orc.skron(G, H) @ orc.svec(A)
    rhs = 0.5 * orc.svec(H @ A @ G.T + G @ A @ H.T)
    assert np.abs(lhs - rhs).max() < 1e-12


# ---------------------------------------------------------------------------
# interior point methods (App. B.1, B.2)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_ipm_linear_matches_extreme_points(seed):
    """min g1's + eta g2 over {eta>=0, S PSD, eta + tr S <= 1} = min(0, g2, lambda_min(smat g1))."""
    rng = np.random.default_rng(seed)
    k = 4
    G = rng.standard_normal((k, k)); G = G + G.T
    g2 = rng.standard_normal()
    val, S, eta = orc.ipm_linear(orc.svec(G), g2, k)
    ref = min(0.0, g2, orc.jacobi_eigh(G)[0][-1])
    assert abs(val - ref) < 1e-6


def _kkt_check(qp, st, k):
    F1, F2 = orc.qp_residuals(qp, st)
    assert np.abs(F1).max() < 1e-6 and abs(F2) < 1e-6
    assert orc.jacobi_eigh(st.S)[0][-1] > -1e-12 and orc.jacobi_eigh(st.T)[0][-1] > -1e-12
    slack = 1 - np.trace(st.S) - st.eta
    assert st.eta >= 0 and slack >= -1e-12 and st.zeta >= 0 and st.omega >= 0
    gapc = np.sum(st.S * st.T) + st.eta * st.zeta + st.omega * slack
    # stop rule mu < 1e-7 with mu = min(mu_prev, gamma gap / (2(k+2))), gamma >= 0.1
    assert gapc < 20 * (k + 2) * 1e-7


def _random_qp(k, rng, m=30):
    d = k * (k + 1) // 2
    Gm = rng.standard_normal((m, d))
    Q11 = Gm.T @ Gm
    zb = rng.standard_normal(m)
    return orc.QPData(Q11=Q11, q12=Gm.T @ zb, q22=float(zb @ zb), h1=rng.standard_normal(d) * 3,
                      h2=rng.standard_normal() * 3)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_ipm_qsdp_kkt(seed):
    """The IPM output satisfies the KKT system of the dual barrier Lagrangian (App. B.2)."""
    rng = np.random.default_rng(seed)
    k = 4
    qp = _random_qp(k, rng)
    st = orc.ipm_qsdp(qp, k)
    _kkt_check(qp, st, k)


def test_ipm_qsdp_k1_bruteforce():
    """k = 1: a convex quadratic over the triangle {s >= 0, eta >= 0, s + eta <= 1}; compare
    with an exhaustive search over a fine grid refined around the best point."""
    rng = np.random.default_rng(7)
    for _ in range(3):
        qp = _random_qp(1, rng, m=3)
        st = orc.ipm_qsdp(qp, 1)
        f = lambda s, e: 0.5 * qp.Q11[0, 0] * s * s + e * qp.q12[0] * s + 0.5 * qp.q22 * e * e \
            + qp.h1[0] * s + qp.h2 * e
        best, arg = np.inf, None
        for s in np.linspace(0, 1, 401):
            es = np.linspace(0, 1 - s, 401)
            v = f(s, es)
            i = int(np.argmin(v))
            if v[i] < best:
                best, arg = v[i], (s, es[i])
        fi = f(st.S[0, 0], st.eta)
        assert fi <= best + 20 * 3 * 1e-7    # duality gap bound of the stop rule (k = 1)
        assert fi >= best - 1e-4   # the grid optimum is within grid resolution of the true one


def test_ipm_warm_start_same_solution():
    rng = np.random.default_rng(11)
    k = 3
    qp = _random_qp(k, rng)
    st = orc.ipm_qsdp(qp, k)
    qp2 = orc.QPData(qp.Q11, qp.q12, qp.q22, qp.h1 + 0.01 * rng.standard_normal(qp.h1.size), qp.h2)
    cold = orc.ipm_qsdp(qp2, k)
    warm = orc.ipm_qsdp(qp2, k, start=st)
    # both stop within the duality-gap bound 20 (k+2) mu_stop of the optimum
    assert abs(orc.qp_objective(qp2, cold.S, cold.eta) - orc.qp_objective(qp2, warm.S, warm.eta)) < 20 * (k + 2) * 1e-7


def _fhat_by_ipm(sc, y, V, Xbar, tau, alpha):
    """Model value f^_t(y) (eq. model_def over eq. subspace_def) found by the interior point
    method of App. B.1 instead of the extreme points: maximise <M, eta Xbar/tau + V S V^T>
    over {eta >= 0, S PSD, eta + tr S <= 1}, i.e. minimise its negative."""
    M = sc.C - orc.A_adjoint(sc.prob, y)
    g1 = -orc.svec(V.T @ M @ V)
    g2 = -float(np.sum(M * Xbar)) / tau if tau > 0 else 0.0
    val, _, _ = orc.ipm_linear(g1, g2, V.shape[1], tol_mu=1e-12)
    return alpha * (-val) + float(sc.b @ y)


def test_fhat_closed_form_equals_ipm_along_a_run():
    """At every iteration of a planted run the closed form of f^_t(y~) equals the App. B.1 IPM
    on the same (V, Xbar, tau, y~).  Early iterations have lambda_max(V^T M V) far below
    lambda_max(M), so using the latter in the closed form fails here."""
    prob = si.maxcut_planted_pm1(40, 5.0, seed=1)
    prm = orc.Params(rho=0.1)
    sc = orc.scale_problem(prob)
    Psi = si.test_matrix(prob.n, 10, seed=0).astype(float)
    st = orc.cold_start(sc, prm, Psi)
    separated = 0
    for _ in range(25):
        V, Xbar, tau = st.V.copy(), st.Xbar.copy(), st.tau
        rec = orc.usbs_step(sc, prm, st, Psi)
        y = rec["y_cand"]
        ref = _fhat_by_ipm(sc, y, V, Xbar, tau, prm.alpha)
        assert abs(rec["fhat"] - ref) <= 1e-8, (rec["fhat"], ref)
        M = sc.C - orc.A_adjoint(prob, y)
        separated += orc.jacobi_eigh(M)[0][0] - orc.jacobi_eigh(V.T @ M @ V)[0][0] > 1e-3
    assert separated >= 2


@pytest.mark.parametrize("case", ["xbar_on_top", "v_misses_top"])
def test_fhat_closed_form_extreme_cases(case):
    """Constructed models where each term of the closed form decides the value alone.
    xbar_on_top: Xbar is a multiple of the top eigenvector's projector and V is orthogonal
    to it, so <M, Xbar>/tau > lambda_max(V^T M V) (dropping the Xbar term fails).
    v_misses_top: Xbar = 0 and V misses the top eigenvector, so lambda_max(V^T M V) <
    lambda_max(M) (using the full spectrum fails)."""
    prob = si.maxcut_er(30, 0.3, seed=5)
    sc = orc.scale_problem(prob)
    rng = np.random.default_rng(9)
    y = 0.02 * rng.standard_normal(prob.m)
    M = sc.C - orc.A_adjoint(prob, y)
    w, Q = orc.jacobi_eigh(M)
    k = 4
    V = Q[:, 3:3 + k] if case == "v_misses_top" else Q[:, 5:5 + k]
    if case == "xbar_on_top":
        tau = 2.7
        Xbar = tau * np.outer(Q[:, 0], Q[:, 0])
        assert float(np.sum(M * Xbar)) / tau > orc.jacobi_eigh(V.T @ M @ V)[0][0] + 1e-3
    else:
        tau, Xbar = 0.0, np.zeros_like(M)
        assert w[0] > orc.jacobi_eigh(V.T @ M @ V)[0][0] + 1e-3
    cf = orc.fhat_closed_form(sc, y, V, Xbar, tau, 2.0)
    assert abs(cf - _fhat_by_ipm(sc, y, V, Xbar, tau, 2.0)) <= 1e-8


def _psi_t(sc, X, y, w, rho):
    """psi_t(X, nu) of Sec. 3.2 with w = b - nu, from its definition on a formed X."""
    AX = orc.A_apply(sc.prob, X)
    r = w - AX
    return float(np.sum(sc.C * X)) + float(r @ y) - float(r @ r) / (2.0 * rho)


@pytest.mark.parametrize("kind", ["maxcut", "cc"])
def test_qp_data_is_negated_psi_t(kind):
    """App. B.2: the master QP is the maximisation of psi_t over the model's set, written in
    (eta, S) with X = alpha((eta/tau) Xbar + V S V^T).  So the QP objective plus psi_t of that X
    is the same constant for every (eta, S); with tau != 1 a wrong power of tau in q12, q22 or
    h2, a dropped term or a wrong sign changes it from one (eta, S) to the next."""
    prob = si.maxcut_er(24, 0.3, seed=4) if kind == "maxcut" else si.cc_signed(24, avg_degree=4, seed=2)
    sc = orc.scale_problem(prob)
    rng = np.random.default_rng(13)
    n, k, alpha, rho = prob.n, 3, 2.0, 0.05
    V = np.linalg.qr(rng.standard_normal((n, k)))[0]
    F = rng.standard_normal((n, 5))
    Xbar = F @ F.T
    Xbar *= 3.7 / np.trace(Xbar)
    tau = float(np.trace(Xbar))
    y = rng.standard_normal(prob.m)
    nu = np.where(prob.is_ineq.astype(bool), np.abs(rng.standard_normal(prob.m)), 0.0)
    w = sc.b - nu
    qp = orc.qp_data(sc, V, orc.constraint_blocks(prob, V), V.T @ sc.C @ V, y, w,
                     orc.A_apply(prob, Xbar), float(np.sum(sc.C * Xbar)), tau, alpha, rho)
    consts = []
    for _ in range(4):
        G = rng.standard_normal((k, k))
        S = G @ G.T
        s_tr, eta = rng.uniform(0.1, 0.6), rng.uniform(0.05, 0.35)
        S *= s_tr / np.trace(S)
        X = alpha * ((eta / tau) * Xbar + V @ S @ V.T)
        consts.append(orc.qp_objective(qp, S, eta) + _psi_t(sc, X, y, w, rho))
    scale = max(1.0, max(abs(c) for c in consts))
    assert max(consts) - min(consts) <= 1e-10 * scale, consts
    # the constant itself: psi_t at X = 0 is <w, y> - ||w||^2 / (2 rho), the QP objective 0
    assert abs(consts[0] - (float(w @ y) - float(w @ w) / (2 * rho))) <= 1e-10 * scale


# ---------------------------------------------------------------------------
# Nystrom sketch (Sec. 4, App. C.1)
# ---------------------------------------------------------------------------
def test_nystrom_exact_for_low_rank():
    rng = np.random.default_rng(3)
    n, r = 60, 10
    F = rng.standard_normal((n, 6))
    X = F @ F.T
    Psi = si.test_matrix(n, r, seed=1).astype(float)
    P = X @ Psi
    assert np.abs(orc.nystrom_definition(P, Psi) - X).max() < 1e-9 * np.abs(X).max()
    U, lam = orc.nystrom_stable(P, Psi)
    assert np.abs((U * lam) @ U.T - X).max() < 1e-9 * np.abs(X).max()
    assert np.abs(U.T @ U - np.eye(r)).max() < 1e-10


def test_nystrom_error_bound_fact_c1():
    """E ||X - Xhat||_* <= (1 + r'/(r - r' - 1)) ||X - [[X]]_r'||_* (Fact C.1), averaged over seeds."""
    rng = np.random.default_rng(4)
    n, r, rp = 50, 10, 4
    Q = np.linalg.qr(rng.standard_normal((n, n)))[0]
    ev = 0.6 ** np.arange(n)
    X = (Q * ev) @ Q.T
    tail = ev[rp:].sum()
    errs = []
    for s in range(30):
        Psi = si.test_matrix(n, r, seed=100 + s).astype(float)
        U, lam = orc.nystrom_stable(X @ Psi, Psi)
        E = X - (U * lam) @ U.T
        errs.append(np.abs(orc.jacobi_eigh(0.5 * (E + E.T))[0]).sum())
    assert np.mean(errs) <= (1 + rp / (r - rp - 1)) * tail


# ---------------------------------------------------------------------------
# operators and scaling
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kind", ["cc", "overlap"])
def test_adjoint_identity_and_lowrank(kind):
    """<A X, y> = <X, A^* y>, and A on low-rank factors equals A on the formed matrix; the
    overlap case has off-diagonal pairs shared by up to eight rows.  The bounds are absolute:
    at these sizes (|X_ij| <= 7, |<A X, y>| <= 15) both identities hold to about 1e-15, so
    nothing is gained by a bound relative to the magnitude."""
    prob = si.cc_signed(30, avg_degree=4, seed=1) if kind == "cc" else si.general_overlap(60, seed=2)
    rng = np.random.default_rng(5)
    F = rng.standard_normal((prob.n, 3))
    lam = rng.random(3)
    X = (F * lam) @ F.T
    y = rng.standard_normal(prob.m)
    assert abs(orc.A_apply(prob, X) @ y - np.sum(X * orc.A_adjoint(prob, y))) < 1e-10
    assert np.abs(orc.A_lowrank(prob, F, lam) - orc.A_apply(prob, X)).max() < 1e-12
    # a row's value is the sum of its triplets written out entry by entry
    k = prob.n + 3 if kind == "overlap" else prob.n
    sel = prob.a_row == k
    direct = sum(v * X[i, j] for i, j, v in zip(prob.a_i[sel], prob.a_j[sel], prob.a_v[sel]))
    assert abs(orc.A_apply(prob, X)[k] - direct) < 1e-12


def test_scaling_units():
    prob = si.maxcut_er(40, 0.2, seed=2)
    sc = orc.scale_problem(prob)
    assert abs(np.linalg.norm(sc.C) - 1) < 1e-12
    assert abs(sc.b.sum() - 1) < 1e-12          # tr X* = 1 after scaling (diag X = 1/n)
    assert np.allclose(orc.dense_C(prob), orc.dense_C(prob).T)


def test_dual_bound_eigenvalue():
    """For MaxCut y = (lambda_max(L)/4) 1 is dual feasible: p* <= (n/4) lambda_max(L); f(y) >= p*."""
    prob = si.maxcut_er(30, 0.3, seed=3)
    sc = orc.scale_problem(prob)
    L4 = orc.dense_C(prob)
    lmax = orc.jacobi_eigh(L4)[0][0]
    y_orig = lmax * np.ones(prob.n)
    f, _, _ = orc.penalized_dual(sc, y_orig / sc.sigma, 2.0, 1)
    assert abs(orc.to_original(sc, f) - prob.n * lmax) < 1e-9 * prob.n * lmax


# ---------------------------------------------------------------------------
# full USBS runs against closed-form SDP values
# ---------------------------------------------------------------------------
def _solve(prob, eps=1e-3, rho=0.1, iters=800, kc=10, kp=1):
    prm = orc.Params(rho=rho, eps_gap=eps, eps_infeas=eps, max_iters=iters, k_c=kc, k_p=kp)
    psi = si.test_matrix(prob.n, 10, seed=0)
    res = orc.usbs_solve(prob, prm, Psi=psi)
    sc = orc.scale_problem(prob)
    return res, sc


def test_usbs_complete_graph():
    """K_n: X = (n/(n-1))(I - J/n) and y = (n/4) 1 give p* = d* = n^2/4."""
    n = 12
    prob = si.maxcut_problem(n, *si.complete_graph(n), np.ones(n * (n - 1) // 2))
    res, sc = _solve(prob)
    assert res.converged
    p = orc.to_original(sc, res.primal_obj)
    f = orc.to_original(sc, res.f)
    assert f >= n * n / 4 - 1e-9            # f(y) >= p* for every y
    assert abs(p - n * n / 4) / (n * n / 4) < 5e-3
    assert abs(f - n * n / 4) / (n * n / 4) < 5e-3


def test_usbs_bipartite_and_odd_cycle():
    """Even cycle: p* = |E|.  Odd cycle C_5: p* = (5/2)(1 + cos(pi/5)) = (25 + 5 sqrt 5)/8."""
    for n, pstar in ((8, 8.0), (5, (25 + 5 * math.sqrt(5)) / 8)):
        i, j = si.cycle_graph(n)
        prob = si.maxcut_problem(n, i, j, np.ones(n))
        res, sc = _solve(prob, kc=3, kp=1)
        f = orc.to_original(sc, res.f)
        p = orc.to_original(sc, res.primal_obj)
        assert f >= pstar - 1e-9
        assert abs(f - pstar) / pstar < 5e-3 and abs(p - pstar) / pstar < 5e-3, (n, p, f, pstar)


def test_usbs_planted_signed_graph_and_invariants():
    """Planted +-1 graph: p* = #positive edges.  Along the run: f(y_t) non-increasing, the model
    is a minorant f^_t(y~) <= f(y~), tr X_{t+1} <= alpha, X_{t+1} PSD, tracked quantities equal
    their dense recomputation."""
    prob = si.maxcut_planted_pm1(40, 5.0, seed=1)
    pstar = prob.meta["p_star"]
    prm = orc.Params(rho=0.1, max_iters=300)
    sc = orc.scale_problem(prob)
    Psi = si.test_matrix(prob.n, 10, seed=0).astype(float)
    st = orc.cold_start(sc, prm, Psi)
    fprev = st.f
    for t in range(300):
        V, Xbar, tau = st.V.copy(), st.Xbar.copy(), st.tau
        rec = orc.usbs_step(sc, prm, st, Psi)
        assert rec["f"] <= fprev + 1e-15
        fprev = rec["f"]
        assert rec["fhat"] <= rec["f_cand"] + 1e-6
        S, eta = st.ipm.S, st.ipm.eta
        g = prm.alpha * eta / tau if tau > 0 else 0.0
        X = g * Xbar + prm.alpha * V @ S @ V.T
        assert np.trace(X) <= prm.alpha + 1e-9
        assert orc.jacobi_eigh(X)[0][-1] > -1e-9
        assert abs(np.trace(st.Xbar) - st.tau) < 1e-12
        assert abs(np.sum(sc.C * st.Xbar) - st.cbar) < 1e-12
        assert np.abs(orc.A_apply(prob, st.Xbar) - st.zbar).max() < 1e-12
        assert np.abs(st.Xbar @ Psi - st.Pbar).max() < 1e-11
        if rec["rel_gap"] <= 1e-3 and rec["rel_infeas"] <= 1e-3:
            break
    p = orc.to_original(sc, rec["primal"])
    f = orc.to_original(sc, rec["f"])
    assert f >= pstar - 1e-9
    assert abs(p - pstar) / pstar < 5e-3 and abs(f - pstar) / pstar < 5e-3


def test_usbs_bruteforce_cut_and_gw_bound():
    """Tiny random graphs: cut* <= p_SDP <= f(y) and, for w >= 0, cut* >= 0.87856 p_SDP."""
    for seed in range(2):
        prob = si.maxcut_er(12, 0.4, seed=seed)
        i, j, w = prob.meta["edges_i"], prob.meta["edges_j"], prob.meta["weights"]
        cut = orc.brute_force_maxcut(prob.n, i, j, w)
        res, sc = _solve(prob, kc=5, kp=1)
        f = orc.to_original(sc, res.f)
        p = orc.to_original(sc, res.primal_obj)
        assert cut <= f + 1e-9
        assert cut >= 0.87856 * p * (1 - 2e-3)


def test_usbs_cc_closed_forms():
    """Correlation clustering: W >= 0 gives X = J, p* = sum_ij W_ij.  Two planted clusters with
    positive weights inside and negative weights across give X = blockdiag(J, J) (|X_ij| <= 1 and
    X_ij >= 0 bound every term), p* = 2 x the within-cluster weight."""
    rng = np.random.default_rng(3)
    n = 16
    i, j = si.random_edges(n, 40, rng)
    w = 0.5 + rng.random(i.size)
    side = np.arange(n) < n // 2
    w2 = np.where(side[i] == side[j], w, -w)
    for ww, pstar in ((w, 2 * w.sum()), (w2, 2 * w2[side[i] == side[j]].sum())):
        prob = si.cc_problem(n, i, j, ww)
        res, sc = _solve(prob, kc=3, kp=0, iters=600)
        f = orc.to_original(sc, res.f)
        p = orc.to_original(sc, res.primal_obj)
        assert res.converged
        assert f >= pstar - 1e-9
        assert abs(p - pstar) / pstar < 1e-2 and abs(f - pstar) / pstar < 1e-2, (p, f, pstar)
        assert np.all(res.y[prob.is_ineq.astype(bool)] >= 0)


def test_oracle_warm_start_grown_problem():
    """Warm start after adding 1% vertices (Sec. 5.1): the padded state is consistent (tracked
    quantities equal the dense recomputation), and the warm solve converges to the cold value."""
    import sdp_inputs as si2
    rng = np.random.default_rng(8)
    n0, n = 60, 61
    i, j = si2.erdos_renyi(n, 0.15, rng)
    keep = (i < n0) & (j < n0)
    base = si2.maxcut_problem(n0, i[keep], j[keep], np.ones(int(keep.sum())))
    grown = si2.maxcut_problem(n, i, j, np.ones(i.size))
    psi0 = si2.test_matrix(n0, 10, seed=2).astype(float)
    psi1 = si2.test_matrix(n, 10, seed=2).astype(float)
    assert np.array_equal(psi1[:n0], psi0)
    prm = orc.Params(rho=0.1, max_iters=600)
    r0 = orc.usbs_solve(base, prm, Psi=psi0)
    assert r0.converged
    sc0 = orc.scale_problem(base)
    sc1, st = orc.warm_start(grown, prm, sc0, r0.state, psi0, psi1)
    assert abs(st.tau - np.trace(st.Xbar)) < 1e-12 and np.abs(st.Pbar - st.Xbar @ psi1).max() < 1e-12
    assert np.abs(st.V.T @ st.V - np.eye(st.V.shape[1])).max() < 1e-12
    warm = orc.usbs_solve(grown, prm, Psi=psi1, state=st)
    cold = orc.usbs_solve(grown, prm, Psi=psi1)
    assert warm.converged and cold.converged
    pw, pc = orc.to_original(sc1, warm.primal_obj), orc.to_original(sc1, cold.primal_obj)
    assert abs(pw - pc) / abs(pc) < 5e-3


def test_oracle_lanczos_vs_jacobi_and_closed_form():
    """The plain Lanczos of the certificate evaluator: equals Jacobi's lambda_max on small
    problems; on large bipartite d-regular graphs lambda_max(L/4 - (d/2) I) = 0 exactly."""
    prob = si.cc_signed(300, avg_degree=6, seed=3)
    rng = np.random.default_rng(4)
    y = rng.standard_normal(prob.m) * 0.01
    sc = orc.scale_problem(prob)
    ref = orc.jacobi_eigh(sc.C - orc.A_adjoint(prob, y))[0][0]
    lam, res = orc.lanczos_lambda_max(orc.sparse_shifted(prob, y), steps=300)
    assert abs(lam - ref) < 1e-10 * max(1, abs(ref))
    big = si.maxcut_regular(20000, 4, seed=1, bipartite=True)
    sigma = float(np.linalg.norm(big.val))
    # L/4 of a bipartite d-regular graph has lambda_max = 2d/4 = d/2, so with y_s = (d/2)/sigma
    # the shifted operator C_s - Diag(y_s) has lambda_max = 0 and f(y) = <b, y> = |E| = p*
    y = np.full(big.n, (4 / 2) / sigma)
    lam, res = orc.lanczos_lambda_max(orc.sparse_shifted(big, y), steps=150)
    assert abs(lam) < 1e-6 / sigma and lam <= 1e-9
    cert = orc.certificate(big, y, np.ones(big.n) / big.n, 2.0 * big.n / (sigma * big.n))
    assert abs(cert["f"] * sigma * big.n - 2 * big.n) < 1e-6 * big.n


def test_decoupled_rows_direct_sum():
    """Rows with no off-diagonal coupling (isolated vertices; a zero-weight edge that still
    carries an X_ij >= 0 row is coupled) are found from the edge list independently, and
    lambda_max of the direct sum equals numpy's dense eigvalsh, also when an isolated row
    holds the top eigenvalue (a Krylov run from a generic start cannot see e_i there)."""
    rng = np.random.default_rng(11)
    n, core = 220, 160
    ei, ej = si.random_edges(core, 500, rng)
    w = rng.choice([-1.0, 1.0], size=ei.size)
    mc = si.maxcut_problem(n, ei, ej, w)
    deg = np.bincount(np.concatenate([ei, ej]), minlength=n)
    assert np.array_equal(orc.decoupled_rows(mc), deg == 0)
    sigma = float(np.linalg.norm(mc.val))
    for lift in (0.0, 5.0):
        y = rng.standard_normal(n) * 0.01 / sigma
        y[core + 7] = -lift / sigma          # d_i = -y_i: the top eigenvalue when lifted
        dense = np.linalg.eigvalsh(orc.sparse_shifted(mc, y).toarray())[-1]
        assert abs(orc.lambda_max_sparse(mc, y) - dense) <= 1e-10 * max(1.0, abs(dense))
        c1 = orc.certificate(mc, y, np.zeros(n), 0.0, dense=True)
        c2 = orc.certificate(mc, y, np.zeros(n), 0.0, dense=False)
        assert abs(c1["f"] - c2["f"]) <= 1e-10 * max(1.0, abs(c1["f"]))
    # correlation clustering: an edge of weight 0 keeps its endpoints coupled via X_ij >= 0
    ci, cj = np.array([0, 2, 3]), np.array([1, 5, 4])
    cc = si.cc_problem(8, ci, cj, np.array([1.0, 0.0, -1.0]))
    iso = orc.decoupled_rows(cc)
    assert np.array_equal(np.flatnonzero(iso), [6, 7])


# ---------------------------------------------------------------------------
# certificates of results computed elsewhere (Sec. 5, App. C)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kind,k_p", [("maxcut", 1), ("cc", 0), ("maxcut", 3)])
def test_primal_from_model_update_equals_dense_X(kind, k_p):
    """A X_{t+1} and <C_s, X_{t+1}> rebuilt from the state after the model update (the
    tracked zbar_{t+1}, cbar_{t+1}, the bundle V_t and the QP solution S) equal the same
    quantities of the dense X_{t+1} = g Xbar_t + alpha V_t S V_t^T along an oracle run.
    Dropping the top-k_p part, or taking the k_p smallest eigenpairs instead, fails."""
    prob = si.maxcut_er(50, 0.15, seed=2) if kind == "maxcut" else si.cc_signed(40, avg_degree=6.0, seed=1)
    k_c = 4 if kind == "cc" else 6
    prm = orc.Params(rho=0.1, k_c=k_c, k_p=k_p, max_iters=40)
    sc = orc.scale_problem(prob)
    Psi = si.test_matrix(prob.n, 10, seed=0).astype(float)
    st = orc.cold_start(sc, prm, Psi)
    checked = 0
    for t in range(12):
        V, Xbar, tau = st.V.copy(), st.Xbar.copy(), st.tau
        rec = orc.usbs_step(sc, prm, st, Psi)
        S, eta = st.ipm.S, st.ipm.eta
        g = prm.alpha * eta / tau if tau > 0 else 0.0
        X = g * Xbar + prm.alpha * V @ S @ V.T
        AX, cX = orc.primal_from_model_update(prob, st.zbar, st.cbar, V, S, prm.alpha, k_p)
        ref_AX = orc.A_apply(prob, X)
        assert np.abs(AX - ref_AX).max() <= 1e-12 * (1 + np.abs(ref_AX).max())
        assert abs(cX - float(np.sum(sc.C * X))) <= 1e-12
        assert np.abs(AX - rec["AX"]).max() <= 1e-12 and abs(cX - rec["primal"]) <= 1e-12
        lam = orc.jacobi_eigh(prm.alpha * S)[0]
        if k_p > 0 and lam[0] > 1e-8 * max(1.0, abs(lam[0])):
            # the top-k_p part is what separates X_{t+1} from Xbar_{t+1}
            assert np.abs(orc.A_apply(prob, st.Xbar) - ref_AX).max() > 1e-9
            checked += 1
    if k_p > 0:
        assert checked > 0


def test_sketch_certificate_equals_dense_definition():
    """<C, Xhat> and dist(A Xhat, K) / (1 + ||b||) of Xhat = U diag(lam) U^T match the dense
    definitions (scaled and original units; equality and inequality rows)."""
    rng = np.random.default_rng(4)
    for prob in (si.maxcut_er(60, 0.1, seed=3), si.cc_signed(50, avg_degree=6.0, seed=2)):
        U = rng.standard_normal((prob.n, 5))
        lam = rng.random(5) * 3.0
        X = (U * lam[None, :]) @ U.T
        C = orc.dense_C(prob)
        cx, inf_s = orc.sketch_certificate(prob, U, lam, "scaled")
        _, inf_o = orc.sketch_certificate(prob, U, lam, "original")
        assert abs(cx - float(np.sum(C * X))) <= 1e-10 * (1 + abs(cx))
        z = orc.A_apply(prob, X)
        ineq = prob.is_ineq.astype(bool)
        e = np.where(ineq, np.maximum(z - prob.b, 0.0), z - prob.b)
        assert abs(inf_o - np.linalg.norm(e) / (1 + np.linalg.norm(prob.b))) <= 1e-12
        es = e / prob.trace
        assert abs(inf_s - np.linalg.norm(es) / (1 + np.linalg.norm(prob.b / prob.trace))) <= 1e-12
        if ineq.any():
            assert np.any(e[ineq] == 0.0) or np.all(z[ineq] > prob.b[ineq])


# ---------------------------------------------------------------------------
# test matrix from a seed (Sec. 4): Philox4x32-10 and the Box-Muller map
# ---------------------------------------------------------------------------
def test_philox_known_answers():
    """The three known-answer vectors published with Philox4x32-10 (Random123: zero counter
    and key, all-ones counter and key, and the digits-of-pi counter and key)."""
    kat = [((0, 0, 0, 0), (0, 0), (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)),
           ((0xffffffff,) * 4, (0xffffffff,) * 2, (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)),
           ((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344), (0xa4093822, 0x299f31d0),
            (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1))]
    for ctr, key, expect in kat:
        out = orc.philox4x32_10([np.uint64(x) for x in ctr], [np.uint64(x) for x in key])
        assert [int(v) for v in out] == list(expect)


def test_psi_from_seed_is_standard_normal_and_row_local():
    """Entries are i.i.d. N(0, 1): moments and a Kolmogorov-Smirnov test on 2e5 draws,
    no correlation between paired columns (the cos / sin halves of one Box-Muller pair),
    seeds give different matrices, and a row depends only on (seed, row) (a grown problem
    keeps its first rows)."""
    from scipy import stats
    psi = orc.psi_from_seed(20000, 10, seed=5).astype(np.float64)
    z = psi.ravel()
    assert abs(z.mean()) < 0.01 and abs(z.var() - 1.0) < 0.02
    assert stats.kstest(z, "norm").pvalue > 1e-3
    assert abs(np.corrcoef(psi[:, 0], psi[:, 1])[0, 1]) < 0.03
    assert abs(np.corrcoef(psi[:, 2], psi[:, 5])[0, 1]) < 0.03
    assert np.array_equal(orc.psi_from_seed(300, 10, seed=5), psi[:300])
    assert not np.array_equal(orc.psi_from_seed(300, 10, seed=6), psi[:300])
    # one entry by hand from its definition
    w = orc.philox4x32_10([np.uint64(7), np.uint64(0), np.uint64(1), np.uint64(0)], [np.uint64(5), np.uint64(0)])
    u1 = ((((int(w[1]) << 32) | int(w[0])) >> 11) + 1) * 2.0 ** -53
    u2 = (((int(w[3]) << 32) | int(w[2])) >> 11) * 2.0 ** -53
    assert psi[7, 3] == np.float32(math.sqrt(-2 * math.log(u1)) * math.sin(2 * math.pi * u2))
