"""CPU oracle for Unified Spectral Bundling with Sketching (USBS), FP64.

TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library imports, links or calls
this module: only tests/, __graft_entry__.smoke() and the cpu_baseline leg of
bench.py may use it.  It shares no code with the HIP path; both read their
inputs from the seeded generators in sdp_inputs.

It is a plain, slow, dense implementation, written to be checked against the
paper by eye:
  * problem scaling                                   App. E, eq. std_scaling
  * penalized dual f(y)                               Sec. 3, eq. pen-D
  * model value f^_t(y~) (closed form, and the IPM)   Sec. 3.1 eq. model_def, App. B.1
  * master QP data and its interior point method     App. B.2, eq. compressed_subprob_2
  * alternating maximisation over (X, nu)             Sec. 3.2, eqs. small_quad_sdp, dual_slack_update
  * candidate iterate                                 Sec. 3.2, eq. dual_update
  * descent / null step                               Alg. 1, eq. descent_cond
  * model update                                      Sec. 3.1, eqs. model_update_eigendecomposition,
                                                      x_bar_def, v_next_def
  * implicit tracking of <C,Xbar>, tr Xbar, A Xbar    App. C (tracking equations)
  * Nystrom sketch and reconstruction                 Sec. 4, App. C.1 eq. nystrom_approx
  * relative suboptimality / infeasibility            Sec. 5, eq. relative_error_tol; App. E eq.
                                                      objective_subopt_upper_bound
Every eigenproblem goes through the cyclic Jacobi routine in jacobi.c.

Readings of passages that are silent, garbled or inconsistent (each one is
also listed in the design notes of the repository):
  R1  slack domain N = {nu_I >= 0, nu_I' = 0}; the printed nu_I <= 0 makes the
      indicator of Y infinite, while the projection form of y~ (Sec. 3.2) and
      y~_I >= 0 need nu_I >= 0.
  R2  QP variables are normalised: X = alpha((eta/tau) Xbar + V S V^T) with
      eta + tr S <= 1, tau = tr Xbar (this is what every coefficient of App. B.2
      encodes); with tau = 0 the eta-terms are zero.
  R3  the printed <C,Xbar> update tr(V^T Q_c^T (C V Q_c Lambda_c)) does not
      type-check; it is read as tr(Lambda_c (V Q_c)^T C (V Q_c)).
  R4  cold start: y0 = 0, V0 = top-k eigenvectors of C - A^* y0, Xbar0 = 0.
  R5  IPM: start S = I/(2k), eta = 1/4, T = I, zeta = omega = 1 (a warm start inside the
      alternating maximisation uses 0.9 x previous solution + 0.1 x this point); step length
      delta = min(1, 0.95 delta_max) with delta_max the largest step keeping
      every variable and the trace slack strictly feasible; stop when
      mu < 1e-7 and the residuals F1, F2 are below 1e-7 (max 100 iterations).
  R6  alternating maximisation stops when nu changes by <= 1e-9 (inf-norm) or
      after 50 passes; a single pass when I is empty.
  R7  eigenvalue ties: descending order, stable by index.
  R8  descent test with '<=' as printed.
  R9  convergence is judged on X_{t+1} = alpha((eta/tau) Xbar_t + V S V^T) and
      f(y_{t+1}); suboptimality uses |f(y) - <C,X>| / (1 + |<C,X>|).
  R10 V_{t+1} = orthonormal basis of [V Q_p, v_1..v_kc] by Householder QR.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def build_jacobi(force: bool = False) -> str:
    """Compile jacobi.c into a shared library next to it (gcc, -O2)."""
    src = os.path.join(_HERE, "jacobi.c")
    out = os.path.join(_HERE, "liboracle_jacobi.so")
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
        tmp = out + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, src, "-lm"])
        os.replace(tmp, out)
    return out


def _lib():
    global _LIB
    if _LIB is None:
        lib = ctypes.CDLL(build_jacobi())
        lib.oracle_jacobi_eigh.restype = ctypes.c_int
        lib.oracle_jacobi_eigh.argtypes = [
            ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
            ctypes.c_int, ctypes.c_double]
        _LIB = lib
    return _LIB


def jacobi_eigh(M: np.ndarray, tol: float = 1e-15, max_sweeps: int = 60):
    """All eigenpairs of the symmetric matrix M, eigenvalues descending.
    Returns (w, V) with M V = V diag(w), V orthogonal (columns = eigenvectors)."""
    M = np.asarray(M, dtype=np.float64)
    n = M.shape[0]
    if n == 0:
        return np.zeros(0), np.zeros((0, 0))
    a = np.ascontiguousarray(0.5 * (M + M.T))
    w = np.empty(n)
    vt = np.empty((n, n))
    sweeps = _lib().oracle_jacobi_eigh(n, a.ctypes.data, w.ctypes.data, vt.ctypes.data,
                                       max_sweeps, tol)
    if sweeps < 0:
        raise RuntimeError("Jacobi did not converge")
    return w, np.ascontiguousarray(vt.T)


# --------------------------------------------------------------------------
# the problem, its operators and its scaling
# --------------------------------------------------------------------------

def dense_C(prob) -> np.ndarray:
    n = prob.n
    C = np.zeros((n, n))
    rows = np.repeat(np.arange(n), np.diff(prob.rowptr))
    np.add.at(C, (rows, prob.col.astype(np.int64)), prob.val)
    return C


def A_apply(prob, X: np.ndarray) -> np.ndarray:
    """(A X)_k = <A_k, X> = sum over the triplets of row k of v * X_ij (Sec. 2.1)."""
    z = np.zeros(prob.m)
    np.add.at(z, prob.a_row.astype(np.int64), prob.a_v * X[prob.a_i, prob.a_j])
    return z


def A_adjoint(prob, y: np.ndarray) -> np.ndarray:
    """A^* y = sum_k y_k A_k as a dense matrix (Sec. 2.1)."""
    n = prob.n
    M = np.zeros((n, n))
    c = y[prob.a_row] * prob.a_v
    diag = prob.a_i == prob.a_j
    np.add.at(M, (prob.a_i[diag], prob.a_i[diag]), c[diag])
    off = ~diag
    np.add.at(M, (prob.a_i[off], prob.a_j[off]), 0.5 * c[off])
    np.add.at(M, (prob.a_j[off], prob.a_i[off]), 0.5 * c[off])
    return M


def A_lowrank(prob, W: np.ndarray, lam: np.ndarray) -> np.ndarray:
    """(A(W diag(lam) W^T))_k: for each triplet (k,i,j,v), v * sum_l lam_l W_il W_jl (App. C)."""
    z = np.zeros(prob.m)
    vals = ((W[prob.a_i] * W[prob.a_j]) * lam[None, :]).sum(axis=1)
    np.add.at(z, prob.a_row.astype(np.int64), prob.a_v * vals)
    return z


def proj_K(prob, z: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Projection onto K = {z : z_I <= b_I, z_I' = b_I'} (Sec. 2.1)."""
    ineq = prob.is_ineq.astype(bool)
    return np.where(ineq, np.minimum(z, b), b)


def dist_K(prob, z: np.ndarray, b: np.ndarray) -> float:
    return float(np.linalg.norm(z - proj_K(prob, z, b)))


def proj_Y(prob, y: np.ndarray) -> np.ndarray:
    """Projection onto Y = {y : y_I >= 0} (Sec. 3)."""
    ineq = prob.is_ineq.astype(bool)
    return np.where(ineq, np.maximum(y, 0.0), y)


@dataclass
class Scaled:
    """The problem scaled so that ||C||_F = tr(X*) = 1 (App. E, eq. std_scaling)."""
    prob: object
    C: np.ndarray        # dense C / sigma
    b: np.ndarray        # b / tau_star
    sigma: float         # ||C||_F of the original
    tau_star: float      # tr X* of the original


def scale_problem(prob) -> Scaled:
    sigma = float(np.linalg.norm(prob.val))
    if sigma == 0.0:
        sigma = 1.0
    C = dense_C(prob) / sigma
    return Scaled(prob=prob, C=C, b=prob.b / prob.trace, sigma=sigma, tau_star=float(prob.trace))


# --------------------------------------------------------------------------
# svec, U and the symmetric Kronecker product (App. B)
# --------------------------------------------------------------------------

def svec(A: np.ndarray) -> np.ndarray:
    """Column-wise lower triangle, off-diagonal entries times sqrt(2)."""
    k = A.shape[0]
    out = []
    for j in range(k):
        out.append(A[j, j])
        for i in range(j + 1, k):
            out.append(np.sqrt(2.0) * A[i, j])
    return np.array(out)


def smat(s: np.ndarray, k: int) -> np.ndarray:
    A = np.zeros((k, k))
    p = 0
    for j in range(k):
        A[j, j] = s[p]
        p += 1
        for i in range(j + 1, k):
            A[i, j] = A[j, i] = s[p] / np.sqrt(2.0)
            p += 1
    return A


def svec_U(k: int) -> np.ndarray:
    """U in R^{k(k+1)/2 x k^2} with U vec(A) = svec(A), vec stacking columns (App. B)."""
    d = k * (k + 1) // 2
    U = np.zeros((d, k * k))
    p = 0
    for j in range(k):
        for i in range(j, k):
            if i == j:
                U[p, j * k + i] = 1.0
            else:
                U[p, j * k + i] = 1.0 / np.sqrt(2.0)   # a_ij in vec: column j, row i
                U[p, i * k + j] = 1.0 / np.sqrt(2.0)   # a_ji
            p += 1
    return U


def skron(G: np.ndarray, H: np.ndarray) -> np.ndarray:
    """G (x)_s H = 1/2 U (G (x) H + H (x) G) U^T (App. B)."""
    U = svec_U(G.shape[0])
    return 0.5 * U @ (np.kron(G, H) + np.kron(H, G)) @ U.T


# --------------------------------------------------------------------------
# penalized dual and the eigen step
# --------------------------------------------------------------------------

def penalized_dual(sc: Scaled, y: np.ndarray, alpha: float, k_vecs: int):
    """f(y) = alpha [lambda_max(C - A^* y)]_+ + <b, y> for y in Y (eq. pen-D).
    Returns f, all eigenvalues (descending) and the top k_vecs eigenvectors."""
    M = sc.C - A_adjoint(sc.prob, y)
    w, V = jacobi_eigh(M)
    f = alpha * max(w[0], 0.0) + float(sc.b @ y)
    return f, w, V[:, :k_vecs]


def fhat_closed_form(sc: Scaled, y: np.ndarray, V: np.ndarray, Xbar: np.ndarray, tau: float,
                     alpha: float) -> float:
    """Model value f^_t(y) for y in Y (eq. model_def with subspace_def): a linear function
    maximised over {eta >= 0, S PSD, eta + tr S <= 1}, whose extreme points are 0,
    Xbar/tau and vv^T with v in range V, hence
        alpha * max{0, lambda_max(V^T M V), <M, Xbar>/tau} + <b, y>,  M = C - A^* y."""
    M = sc.C - A_adjoint(sc.prob, y)
    cands = [0.0, jacobi_eigh(V.T @ M @ V)[0][0]]
    if tau > 0:
        cands.append(float(np.sum(M * Xbar)) / tau)
    return alpha * max(cands) + float(sc.b @ y)


# --------------------------------------------------------------------------
# App. B.1: IPM for the linear small SDP (used only to pin the closed form)
# --------------------------------------------------------------------------

def _max_step_psd(X: np.ndarray, dX: np.ndarray) -> float:
    """Largest a with X + a dX PSD (X positive definite)."""
    L = np.linalg.cholesky(X)
    Li = np.linalg.inv(L)
    w = jacobi_eigh(Li @ dX @ Li.T)[0]
    lo = w[-1]
    return np.inf if lo >= 0 else -1.0 / lo


def _max_step_pos(x: float, dx: float) -> float:
    return np.inf if dx >= 0 else -x / dx


def ipm_linear(g1: np.ndarray, g2: float, k: int, tol_mu: float = 1e-9, max_iter: int = 200):
    """min g1^T svec(S) + eta g2 s.t. eta >= 0, S PSD, 1 - tr S - eta >= 0
    (eq. compressed_subprob_1) by the primal-dual method of App. B.1.  Its Newton system
    is the one of App. B.2 with Q11 = 0, q12 = 0, q22 = 0, h1 = g1, h2 = g2, so the
    same routine serves.  Returns (value, S, eta)."""
    qp = QPData(np.zeros((len(g1), len(g1))), np.zeros(len(g1)), 0.0, np.asarray(g1, float), float(g2))
    st = ipm_qsdp(qp, k, tol_mu=tol_mu, tol_res=1e-9, max_iter=max_iter)
    return float(qp.h1 @ svec(st.S) + st.eta * qp.h2), st.S, st.eta


# --------------------------------------------------------------------------
# App. B.2: the master QP and its IPM
# --------------------------------------------------------------------------

def constraint_blocks(prob, V: np.ndarray) -> np.ndarray:
    """Rows svec(V^T A_k V), k = 1..m, as an m x k(k+1)/2 matrix."""
    k = V.shape[1]
    G = np.zeros((prob.m, k * (k + 1) // 2))
    for row, i, j, v in zip(prob.a_row, prob.a_i, prob.a_j, prob.a_v):
        ri, rj = V[i], V[j]
        B = v * np.outer(ri, ri) if i == j else 0.5 * v * (np.outer(ri, rj) + np.outer(rj, ri))
        G[row] += svec(B)
    return G


@dataclass
class QPData:
    Q11: np.ndarray
    q12: np.ndarray
    q22: float
    h1: np.ndarray
    h2: float


def qp_data(sc: Scaled, V, Gk, VCV, y, w, zbar, cbar, tau, alpha, rho) -> QPData:
    """Coefficients of eq. compressed_subprob_2 with w = b - nu~ (App. B.2), under the
    normalisation X = alpha((eta/tau) Xbar + V S V^T).  Gk = constraint_blocks(V)."""
    u = y - w / rho
    h1 = alpha * (Gk.T @ u - svec(VCV))
    Q11 = (alpha ** 2 / rho) * (Gk.T @ Gk)
    if tau > 0:
        q12 = (alpha ** 2 / (rho * tau)) * (Gk.T @ zbar)
        q22 = alpha ** 2 * float(zbar @ zbar) / (rho * tau * tau)
        h2 = (alpha / tau) * (float(u @ zbar) - cbar)
    else:
        q12, q22, h2 = np.zeros_like(h1), 0.0, 0.0
    return QPData(Q11, q12, q22, h1, h2)


@dataclass
class IPMState:
    S: np.ndarray
    eta: float
    T: np.ndarray
    zeta: float
    omega: float
    iters: int = 0


def ipm_init(k: int) -> IPMState:
    return IPMState(np.eye(k) / (2 * k), 0.25, np.eye(k), 1.0, 1.0)


def qp_residuals(qp: QPData, st: IPMState):
    k = st.S.shape[0]
    vI = svec(np.eye(k))
    s, t = svec(st.S), svec(st.T)
    F1 = qp.Q11 @ s + st.eta * qp.q12 + qp.h1 - t + st.omega * vI
    F2 = float(qp.q12 @ s) + st.eta * qp.q22 + qp.h2 - st.zeta + st.omega
    return F1, F2


def qp_objective(qp: QPData, S, eta) -> float:
    s = svec(S)
    return float(0.5 * s @ qp.Q11 @ s + eta * qp.q12 @ s + 0.5 * qp.q22 * eta * eta
                 + qp.h1 @ s + qp.h2 * eta)


def ipm_qsdp(qp: QPData, k: int, start: IPMState | None = None, tol_mu: float = 1e-7,
             tol_res: float = 1e-7, max_iter: int = 100) -> IPMState:
    """Primal-dual path following for eq. compressed_subprob_2 (App. B.2).  Newton
    directions from the unreduced linearised system (the five block equations of
    App. B.2) solved by dense LU; mu estimate, step and mu update as in App. B.1."""
    d = k * (k + 1) // 2
    vI = svec(np.eye(k))
    st = ipm_init(k)
    if start is not None:
        # warm start (App. B.2): the previous solution, pulled 10% of the way towards the
        # default interior point so that it is strictly inside the cone again
        a = 0.1
        st = IPMState((1 - a) * start.S + a * st.S, (1 - a) * start.eta + a * st.eta,
                      (1 - a) * start.T + a * st.T, (1 - a) * start.zeta + a * st.zeta,
                      (1 - a) * start.omega + a * st.omega)
    S, eta, T, zeta, om = st.S, st.eta, st.T, st.zeta, st.omega
    slack = 1.0 - np.trace(S) - eta
    mu = (np.sum(S * T) + eta * zeta + om * slack) / (2 * (k + 2))
    it = 0
    for it in range(1, max_iter + 1):
        s, t = svec(S), svec(T)
        F1 = qp.Q11 @ s + eta * qp.q12 + qp.h1 - t + om * vI
        F2 = float(qp.q12 @ s) + eta * qp.q22 + qp.h2 - zeta + om
        if mu < tol_mu and max(np.max(np.abs(F1)), abs(F2)) < tol_res:
            it -= 1
            break
        Si = np.linalg.inv(S)
        kap1 = slack / om
        N = 2 * d + 3
        iS, ie, iT, iz, io = 0, d, d + 1, 2 * d + 1, 2 * d + 2
        J = np.zeros((N, N))
        r = np.zeros(N)
        # Q11 ds + deta q12 - dt + dw vI = -F1
        J[0:d, iS:iS + d] = qp.Q11
        J[0:d, ie] = qp.q12
        J[0:d, iT:iT + d] = -np.eye(d)
        J[0:d, io] = vI
        r[0:d] = -F1
        # q12^T ds + deta q22 - dzeta + dw = -F2
        J[d, iS:iS + d] = qp.q12
        J[d, ie] = qp.q22
        J[d, iz] = -1.0
        J[d, io] = 1.0
        r[d] = -F2
        # kap1 dw - vI^T ds - deta = mu/w + vI^T s + eta - 1
        J[d + 1, io] = kap1
        J[d + 1, iS:iS + d] = -vI
        J[d + 1, ie] = -1.0
        r[d + 1] = mu / om + vI @ s + eta - 1.0
        # (T (x)s S^-1) ds + dt = mu svec(S^-1) - t
        J[d + 2:2 * d + 2, iS:iS + d] = skron(T, Si)
        J[d + 2:2 * d + 2, iT:iT + d] = np.eye(d)
        r[d + 2:2 * d + 2] = mu * svec(Si) - t
        # zeta/eta deta + dzeta = mu/eta - zeta
        J[2 * d + 2, ie] = zeta / eta
        J[2 * d + 2, iz] = 1.0
        r[2 * d + 2] = mu / eta - zeta
        dx = np.linalg.solve(J, r)
        dS, deta, dT = smat(dx[iS:iS + d], k), dx[ie], smat(dx[iT:iT + d], k)
        dzeta, dom = dx[iz], dx[io]
        dmax = min(_max_step_psd(S, dS), _max_step_psd(T, dT), _max_step_pos(eta, deta),
                   _max_step_pos(zeta, dzeta), _max_step_pos(om, dom),
                   _max_step_pos(slack, -np.trace(dS) - deta))
        delta = min(1.0, 0.95 * dmax)
        S = S + delta * dS
        T = T + delta * dT
        S, T = 0.5 * (S + S.T), 0.5 * (T + T.T)
        eta, zeta, om = eta + delta * deta, zeta + delta * dzeta, om + delta * dom
        slack = 1.0 - np.trace(S) - eta
        gam = 1.0 if delta <= 0.2 else 0.5 - 0.4 * delta * delta
        mu = min(mu, gam * (np.sum(S * T) + eta * zeta + om * slack) / (2 * (k + 2)))
    return IPMState(S, eta, T, zeta, om, it)


# --------------------------------------------------------------------------
# Nystrom sketch reconstruction (Sec. 4, App. C.1)
# --------------------------------------------------------------------------

def nystrom_definition(P: np.ndarray, Psi: np.ndarray) -> np.ndarray:
    """Xhat = P (Psi^T P)^+ P^T, dense (eq. nystrom_approx)."""
    B = Psi.T @ P
    return P @ np.linalg.pinv(0.5 * (B + B.T)) @ P.T


def nystrom_stable(P: np.ndarray, Psi: np.ndarray):
    """Rank-r factors U, lam of the Nystrom approximation by the numerically stable
    fixed-rank PSD method of Tropp, Yurtsever, Udell & Cevher (2017): shift by
    nu = sqrt(n) eps(||P||), Cholesky of the shifted core, thin SVD, remove the shift."""
    n, r = P.shape
    nrm = np.linalg.norm(P, 2) if P.size else 0.0
    nu = np.sqrt(n) * np.spacing(nrm) if nrm > 0 else 0.0
    Pn = P + nu * Psi
    B = Psi.T @ Pn
    B = 0.5 * (B + B.T)
    L = np.linalg.cholesky(B)
    F = np.linalg.solve(L, Pn.T).T          # F = Pn L^{-T}
    Uf, sv, _ = np.linalg.svd(F, full_matrices=False)
    lam = np.maximum(sv * sv - nu, 0.0)
    return Uf, lam


# --------------------------------------------------------------------------
# the USBS iteration (Alg. 1)
# --------------------------------------------------------------------------

@dataclass
class Params:
    alpha: float = 2.0
    rho: float = 0.01
    beta: float = 0.25
    k_c: int = 10
    k_p: int = 1
    r: int = 10
    eps_gap: float = 1e-3
    eps_infeas: float = 1e-3
    max_iters: int = 1000
    units: str = "scaled"       # "scaled" (App. E) or "original"


@dataclass
class State:
    y: np.ndarray
    f: float
    V: np.ndarray
    Xbar: np.ndarray
    tau: float
    cbar: float
    zbar: np.ndarray
    Pbar: np.ndarray
    ipm: IPMState | None = None


@dataclass
class Result:
    y: np.ndarray                 # scaled units
    f: float
    primal_obj: float             # <C_s, X_{T}>
    z: np.ndarray                 # A X_T, scaled
    rel_gap: float
    rel_infeas: float
    iters: int
    descents: int
    converged: bool
    state: State
    history: list = field(default_factory=list)
    X: np.ndarray | None = None


def metrics(sc: Scaled, f: float, cX: float, z: np.ndarray, units: str):
    """eq. relative_error_tol with the upper bound of eq. objective_subopt_upper_bound."""
    if units == "original":
        s = sc.sigma * sc.tau_star
        fo, co = s * f, s * cX
        zo, bo = z * sc.tau_star, sc.prob.b
        gap = abs(fo - co) / (1.0 + abs(co))
        inf = dist_K(sc.prob, zo, bo) / (1.0 + np.linalg.norm(bo))
    else:
        gap = abs(f - cX) / (1.0 + abs(cX))
        inf = dist_K(sc.prob, z, sc.b) / (1.0 + np.linalg.norm(sc.b))
    return gap, inf


def cold_start(sc: Scaled, prm: Params, Psi: np.ndarray) -> State:
    n = sc.prob.n
    k = prm.k_c + prm.k_p
    y0 = np.zeros(sc.prob.m)
    f0, _, V0 = penalized_dual(sc, y0, prm.alpha, k)
    return State(y=y0, f=f0, V=V0, Xbar=np.zeros((n, n)), tau=0.0, cbar=0.0,
                 zbar=np.zeros(sc.prob.m), Pbar=np.zeros((n, Psi.shape[1])))


def usbs_step(sc: Scaled, prm: Params, st: State, Psi: np.ndarray) -> dict:
    """One pass of the loop body of Alg. 1; updates st in place and returns a log record."""
    prob = sc.prob
    k = st.V.shape[1]
    alpha, rho = prm.alpha, prm.rho
    ineq = prob.is_ineq.astype(bool)
    V = st.V
    Gk = constraint_blocks(prob, V)
    VCV = V.T @ sc.C @ V
    # alternating maximisation over (X, nu) (eqs. small_quad_sdp, dual_slack_update)
    nu = np.zeros(prob.m)
    ipm = None
    passes = 0
    ipm_iters = 0
    for passes in range(1, 51):
        qp = qp_data(sc, V, Gk, VCV, st.y, sc.b - nu, st.zbar, st.cbar, st.tau, alpha, rho)
        ipm = ipm_qsdp(qp, k, start=ipm)
        ipm_iters += ipm.iters
        g = alpha * ipm.eta / st.tau if st.tau > 0 else 0.0
        AX = g * st.zbar + alpha * (Gk @ svec(ipm.S))
        if not ineq.any():
            break
        nu_new = np.where(ineq, np.maximum(sc.b - AX - rho * st.y, 0.0), 0.0)
        done = np.max(np.abs(nu_new - nu)) <= 1e-9
        nu = nu_new
        if done:
            break
    S, eta = ipm.S, ipm.eta
    g = alpha * eta / st.tau if st.tau > 0 else 0.0
    # X_{t+1} = g Xbar + alpha V S V^T and its tracked quantities
    AX = g * st.zbar + alpha * (Gk @ svec(S))
    cX = g * st.cbar + alpha * float(np.sum(VCV * S))
    # candidate (eq. dual_update; feasible form of Sec. 3.2)
    y_c = proj_Y(prob, st.y - (sc.b - AX) / rho)
    f_c, w_c, vecs = penalized_dual(sc, y_c, alpha, max(prm.k_c, 1))
    fhat = fhat_closed_form(sc, y_c, V, st.Xbar, st.tau, alpha)
    descent = prm.beta * (st.f - fhat) <= st.f - f_c
    if descent:
        st.y, st.f = y_c, f_c
    # model update: eigen-split of alpha S (eq. model_update_eigendecomposition)
    lam, Q = jacobi_eigh(alpha * S)
    Qp, lp = Q[:, :prm.k_p], lam[:prm.k_p]
    Qc, lc = Q[:, prm.k_p:], lam[prm.k_p:]
    Wc = V @ Qc
    Xnew_c = (Wc * lc[None, :]) @ Wc.T
    st.Xbar = g * st.Xbar + Xnew_c                                    # eq. x_bar_def
    st.tau = g * st.tau + float(np.sum(lc))
    st.cbar = g * st.cbar + float(np.sum(lc * np.diag(Qc.T @ VCV @ Qc)))  # reading R3
    st.zbar = g * st.zbar + A_lowrank(prob, Wc, lc)
    st.Pbar = g * st.Pbar + Wc @ (lc[:, None] * (Wc.T @ Psi))           # Sec. 4 sketch update
    newV = np.concatenate([V @ Qp, vecs], axis=1)                       # eq. v_next_def
    st.V = np.linalg.qr(newV)[0] if prm.k_p > 0 else vecs
    st.ipm = ipm
    gap, inf = metrics(sc, st.f, cX, AX, prm.units)
    return {"f": st.f, "f_cand": f_c, "fhat": fhat, "descent": bool(descent), "lambda1": w_c[0],
            "primal": cX, "rel_gap": gap, "rel_infeas": inf, "eta": eta, "trS": float(np.trace(S)),
            "ipm_iters": ipm_iters, "passes": passes, "AX": AX, "y_cand": y_c}


def usbs_solve(prob, prm: Params | None = None, Psi: np.ndarray | None = None, seed: int = 0,
               state: State | None = None, keep_history: bool = True, callback=None) -> Result:
    """Run Alg. 1 until both relative errors are <= eps (or max_iters)."""
    prm = prm or Params()
    sc = scale_problem(prob)
    if Psi is None:
        from sdp_inputs import test_matrix
        Psi = test_matrix(prob.n, prm.r, seed)
    Psi = np.asarray(Psi, dtype=np.float64)
    st = state if state is not None else cold_start(sc, prm, Psi)
    hist = []
    rec = None
    descents = 0
    converged = False
    it = 0
    for it in range(1, prm.max_iters + 1):
        rec = usbs_step(sc, prm, st, Psi)
        descents += rec["descent"]
        if keep_history:
            hist.append({kk: vv for kk, vv in rec.items() if kk not in ("AX", "y_cand")})
        if callback is not None:
            callback(it, rec)
        if rec["rel_gap"] <= prm.eps_gap and rec["rel_infeas"] <= prm.eps_infeas:
            converged = True
            break
    return Result(y=st.y.copy(), f=st.f, primal_obj=rec["primal"], z=rec["AX"],
                  rel_gap=rec["rel_gap"], rel_infeas=rec["rel_infeas"], iters=it,
                  descents=descents, converged=converged, state=st, history=hist)


def warm_start(prob_new, prm: Params, sc_old: Scaled, st_old: State, Psi_old: np.ndarray,
               Psi_new: np.ndarray):
    """Warm start for a grown problem (Sec. 5.1: pad the old solution with zeros and rescale).
    Reading: Xbar_0 is the rank-r Nystrom reconstruction of the old sketch (App. C.1), padded with
    zero rows and rescaled to the new tr X*; y is padded with zeros and rescaled to the new ||C||_F;
    V is padded and re-orthonormalised.  Returns (scaled problem, state)."""
    sc = scale_problem(prob_new)
    n0, n = sc_old.prob.n, prob_new.n
    U, lam = nystrom_stable(st_old.Pbar, np.asarray(Psi_old, dtype=np.float64))
    Up = np.zeros((n, U.shape[1]))
    Up[:n0] = U
    lam = lam * sc_old.tau_star / sc.tau_star
    Xbar = (Up * lam[None, :]) @ Up.T
    y = np.zeros(prob_new.m)
    y[:sc_old.prob.m] = st_old.y * sc_old.sigma / sc.sigma
    Vp = np.zeros((n, st_old.V.shape[1]))
    Vp[:n0] = st_old.V
    V = np.linalg.qr(Vp)[0]
    f, _, _ = penalized_dual(sc, y, prm.alpha, 1)
    st = State(y=y, f=f, V=V, Xbar=Xbar, tau=float(np.trace(Xbar)), cbar=float(np.sum(sc.C * Xbar)),
               zbar=A_apply(prob_new, Xbar), Pbar=Xbar @ np.asarray(Psi_new, dtype=np.float64))
    return sc, st


def to_original(sc: Scaled, value: float) -> float:
    """Objective values in the units of the unscaled problem."""
    return sc.sigma * sc.tau_star * value


# --------------------------------------------------------------------------
# Gaussian test matrix of the sketch from a seed (Sec. 4: Psi has i.i.d. N(0, 1) entries)
# --------------------------------------------------------------------------
_PHILOX_M = (np.uint64(0xD2511F53), np.uint64(0xCD9E8D57))
_PHILOX_W = (np.uint64(0x9E3779B9), np.uint64(0xBB67AE85))
_MASK32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11), elementwise over arrays:
    ctr = four arrays of 32-bit words, key = two; returns the four output words.  Ten
    rounds; before every round but the first the key is bumped by the Weyl constants."""
    c = [np.asarray(x, dtype=np.uint64) & _MASK32 for x in ctr]
    k = [np.asarray(x, dtype=np.uint64) & _MASK32 for x in key]
    for rnd in range(10):
        if rnd > 0:
            k = [(k[0] + _PHILOX_W[0]) & _MASK32, (k[1] + _PHILOX_W[1]) & _MASK32]
        p0 = _PHILOX_M[0] * c[0]
        p1 = _PHILOX_M[1] * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK32
        c = [hi1 ^ c[1] ^ k[0], lo1, hi0 ^ c[3] ^ k[1], lo0]
    return c


def psi_from_seed(n: int, r: int, seed: int) -> np.ndarray:
    """n x r test matrix (float32): entry (i, c) from the Philox block with counter
    (i mod 2^32, i div 2^32, c div 2, 0) and key (seed mod 2^32, seed div 2^32); the words
    give u1 = ((w1 w0 >> 11) + 1) 2^-53 in (0, 1] and u2 = (w3 w2 >> 11) 2^-53 in [0, 1), and the
    Box-Muller pair sqrt(-2 ln u1) (cos 2 pi u2, sin 2 pi u2) gives columns 2q and 2q + 1."""
    i = np.repeat(np.arange(n, dtype=np.uint64), r)
    col = np.tile(np.arange(r, dtype=np.uint64), n)
    seed = np.uint64(seed)
    w = philox4x32_10([i & _MASK32, i >> np.uint64(32), col >> np.uint64(1), np.zeros_like(i)],
                      [seed & _MASK32, seed >> np.uint64(32)])
    a = (w[1] << np.uint64(32)) | w[0]
    b = (w[3] << np.uint64(32)) | w[2]
    u1 = ((a >> np.uint64(11)) + np.uint64(1)).astype(np.float64) * 2.0 ** -53
    u2 = (b >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    rad = np.sqrt(-2.0 * np.log(u1))
    z = np.where((col & np.uint64(1)) == 1, rad * np.sin(2.0 * np.pi * u2), rad * np.cos(2.0 * np.pi * u2))
    return z.astype(np.float32).reshape(n, r)


# --------------------------------------------------------------------------
# certificates for a result computed elsewhere
# --------------------------------------------------------------------------

def sparse_shifted(prob, y_scaled: np.ndarray):
    """C_s - A^* y as a scipy CSR matrix (for n too large for dense storage)."""
    import scipy.sparse as sp
    n = prob.n
    sigma = float(np.linalg.norm(prob.val)) or 1.0
    rows = np.repeat(np.arange(n), np.diff(prob.rowptr))
    M = sp.csr_matrix((prob.val / sigma, (rows, prob.col.astype(np.int64))), shape=(n, n))
    c = y_scaled[prob.a_row] * prob.a_v
    diag = prob.a_i == prob.a_j
    off = ~diag
    Ay = sp.coo_matrix((np.concatenate([c[diag], 0.5 * c[off], 0.5 * c[off]]),
                        (np.concatenate([prob.a_i[diag], prob.a_i[off], prob.a_j[off]]),
                         np.concatenate([prob.a_i[diag], prob.a_j[off], prob.a_i[off]]))), shape=(n, n))
    return (M - Ay.tocsr()).tocsr()


def lanczos_lambda_max(M, steps: int = 200, seed: int = 0):
    """Largest eigenvalue of a symmetric (sparse or dense) matrix by plain single-vector
    Lanczos with full re-orthogonalisation and the Jacobi eigenvalues of the tridiagonal
    matrix; returns (theta_1, residual bound |beta_k y_k1|)."""
    n = M.shape[0]
    steps = min(steps, n)
    rng = np.random.default_rng(seed)
    Q = np.zeros((steps + 1, n))
    q = rng.standard_normal(n)
    Q[0] = q / np.linalg.norm(q)
    alpha, beta = [], []
    k = 0
    for k in range(steps):
        w = M @ Q[k]
        a = float(Q[k] @ w)
        w = w - Q[:k + 1].T @ (Q[:k + 1] @ w)
        w = w - Q[:k + 1].T @ (Q[:k + 1] @ w)
        b = float(np.linalg.norm(w))
        alpha.append(a)
        beta.append(b)
        if b < 1e-14 * max(1.0, abs(a)):
            break
        Q[k + 1] = w / b
    m = len(alpha)
    T = np.diag(alpha) + np.diag(beta[:m - 1], 1) + np.diag(beta[:m - 1], -1)
    w, Y = jacobi_eigh(T)
    return float(w[0]), float(abs(beta[m - 1] * Y[m - 1, 0]))

def decoupled_rows(prob) -> np.ndarray:
    """Mask of the rows i on which C - A^*(y) has no off-diagonal entry whatever y is:
    no nonzero C_ij (j != i) and no constraint with a term in an off-diagonal pair
    (i, j).  On those rows the matrix is diagonal, so it is the direct sum of the
    coupled block and diag(d_i): its spectrum is the coupled block's spectrum together
    with the d_i, and e_i is an exact eigenvector."""
    n = prob.n
    rows = np.repeat(np.arange(n), np.diff(prob.rowptr))
    col = np.asarray(prob.col, dtype=np.int64)
    off = (col != rows) & (np.asarray(prob.val) != 0.0)
    coupled = np.zeros(n, dtype=bool)
    coupled[rows[off]] = True
    t_off = prob.a_i != prob.a_j
    coupled[prob.a_i[t_off]] = True
    coupled[prob.a_j[t_off]] = True
    return ~coupled


def lambda_max_sparse(prob, y_scaled: np.ndarray, steps: int = 300, seed: int = 0) -> float:
    """lambda_max(C_s - A^* y) for n too large for a dense eigensolver: Lanczos on the
    coupled block, and the exact diagonal entries of the decoupled rows (the matrix is
    their direct sum)."""
    M = sparse_shifted(prob, y_scaled)
    iso = decoupled_rows(prob)
    cand = []
    if iso.any():
        cand.append(float(M.diagonal()[iso].max()))
    cpl = np.flatnonzero(~iso)
    if cpl.size:
        cand.append(lanczos_lambda_max(M[cpl][:, cpl], steps=steps, seed=seed)[0])
    return max(cand)


def certificate(prob, y_scaled: np.ndarray, z_scaled: np.ndarray, cX_scaled: float,
                alpha: float = 2.0, units: str = "scaled", lam_max: float | None = None,
                dense: bool | None = None):
    """Re-evaluate f(y) in FP64 and the relative errors of a primal summary (z = A X,
    <C, X>) produced by another solver, all in scaled units.  lambda_max comes from the
    Jacobi eigenvalues of the dense matrix (n <= 3000 unless dense says otherwise) or
    from lambda_max_sparse."""
    if dense is None:
        dense = prob.n <= 3000
    sc = scale_problem(prob) if dense else None
    y = proj_Y(prob, np.asarray(y_scaled, dtype=np.float64))
    if sc is None:
        sigma = float(np.linalg.norm(prob.val)) or 1.0
        sc = Scaled(prob=prob, C=None, b=prob.b / prob.trace, sigma=sigma, tau_star=float(prob.trace))
    if lam_max is None:
        if sc.C is not None:
            lam_max = jacobi_eigh(sc.C - A_adjoint(prob, y))[0][0]
        else:
            lam_max = lambda_max_sparse(prob, y)
    f = alpha * max(lam_max, 0.0) + float(sc.b @ y)
    gap, inf = metrics(sc, f, cX_scaled, np.asarray(z_scaled, dtype=np.float64), units)
    return {"f": f, "lambda_max": lam_max, "rel_gap": gap, "rel_infeas": inf}


def C_quadratic_forms(prob, W: np.ndarray) -> np.ndarray:
    """diag(W^T C_s W) for an n x q block W (C_s = C / ||C||_F, App. E), with C applied
    in its sparse form so that it serves at any n."""
    import scipy.sparse as sp
    n = prob.n
    sigma = float(np.linalg.norm(prob.val)) or 1.0
    rows = np.repeat(np.arange(n), np.diff(prob.rowptr))
    C = sp.csr_matrix((prob.val / sigma, (rows, prob.col.astype(np.int64))), shape=(n, n))
    W = np.asarray(W, dtype=np.float64).reshape(n, -1)
    return np.einsum("iq,iq->q", W, C @ W)


def primal_from_model_update(prob, zbar_next: np.ndarray, cbar_next: float, V: np.ndarray, S: np.ndarray,
                             alpha: float, k_p: int):
    """A X_{t+1} and <C_s, X_{t+1}> of X_{t+1} = alpha((eta/tau) Xbar_t + V S V^T) from the
    tracked quantities after the model update (Sec. 3.1, eqs. model_update_eigendecomposition
    and x_bar_def; App. C tracking).  With alpha S = Q_p Lam_p Q_p^T + Q_c Lam_c Q_c^T (top
    k_p eigenpairs first) the update sets Xbar_{t+1} = (alpha eta/tau) Xbar_t + (V Q_c) Lam_c
    (V Q_c)^T, so X_{t+1} = Xbar_{t+1} + (V Q_p) Lam_p (V Q_p)^T."""
    lam, Q = jacobi_eigh(alpha * np.asarray(S, dtype=np.float64))
    Wp = np.asarray(V, dtype=np.float64) @ Q[:, :k_p]
    lp = lam[:k_p]
    AX = np.asarray(zbar_next, dtype=np.float64) + A_lowrank(prob, Wp, lp)
    cX = float(cbar_next) + float(np.sum(lp * C_quadratic_forms(prob, Wp)))
    return AX, cX


def sketch_certificate(prob, U: np.ndarray, lam: np.ndarray, units: str = "scaled"):
    """<C, Xhat> (original units) and the relative infeasibility of Xhat = U diag(lam) U^T,
    the Nystrom reconstruction handed out in original units (Sec. 4, App. C.1), measured as
    in eq. relative_error_tol: dist(A Xhat, K) / (1 + ||b||) in the chosen units."""
    U = np.asarray(U, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    sigma = float(np.linalg.norm(prob.val)) or 1.0
    cx = sigma * float(np.sum(lam * C_quadratic_forms(prob, U)))
    z = A_lowrank(prob, U, lam)
    if units == "original":
        inf = dist_K(prob, z, prob.b) / (1.0 + np.linalg.norm(prob.b))
    else:
        bs = prob.b / prob.trace
        inf = dist_K(prob, z / prob.trace, bs) / (1.0 + np.linalg.norm(bs))
    return cx, inf


# --------------------------------------------------------------------------
# MaxCut helpers (App. E.1)
# --------------------------------------------------------------------------

def cut_value(i, j, w, x) -> float:
    x = np.asarray(x)
    return float(np.sum(np.asarray(w)[x[i] != x[j]]))


def maxcut_round(U: np.ndarray, i, j, w):
    """Best of the cuts sign(U[:, c]) over the columns c (App. E.1 rounding)."""
    best, best_x = -np.inf, None
    for c in range(U.shape[1]):
        x = U[:, c] >= 0
        v = cut_value(i, j, w, x)
        if v > best:
            best, best_x = v, x
    return best, best_x


def brute_force_maxcut(n: int, i, j, w) -> float:
    """Exact max cut of a tiny graph by enumeration of the 2^(n-1) cuts."""
    i = np.asarray(i)
    j = np.asarray(j)
    w = np.asarray(w, dtype=np.float64)
    best = -np.inf
    chunk = 1 << 16
    for s in range(0, 1 << (n - 1), chunk):
        ids = np.arange(s, min(s + chunk, 1 << (n - 1)))
        x = ((ids[:, None] >> np.arange(n - 1)[None, :]) & 1).astype(np.int8)
        x = np.concatenate([x, np.zeros((x.shape[0], 1), dtype=np.int8)], axis=1)
        vals = ((x[:, i] != x[:, j]) * w[None, :]).sum(axis=1)
        best = max(best, float(vals.max()))
    return best
