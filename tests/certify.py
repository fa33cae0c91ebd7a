"""Oracle certificate of a GPU solve (test helper, imported by the GPU tests).

Everything a GPU result claims is recomputed here by the FP64 oracle from what the
library hands out through the C ABI:
  * f(y) = alpha [lambda_max(C_s - A^* y)]_+ + <b_s, y> from y alone (Jacobi at small n,
    the oracle's Lanczos on the sparse matrix otherwise);
  * A X_{t+1} and <C_s, X_{t+1}> rebuilt from the state after the model update (tracked
    zbar, cbar, the bundle V_t and the QP solution S; Sec. 3.1) and compared with the
    values the library exports (usbs_get_primal);
  * the relative gap and infeasibility of eq. relative_error_tol from those values;
  * <C, Xhat> and the infeasibility of the Nystrom reconstruction Xhat = U diag(lam) U^T
    from the factors usbs_solve returns (Sec. 4, App. C.1).
"""
from __future__ import annotations

import numpy as np

from oracle import usbs_oracle as orc


def certify(prob, solver, out, tol: float = 1e-3, dense: bool | None = None, f_tol: float = 1e-7,
            units: str = "scaled", check_sketch: bool = True, say=print, lanczos_steps: int | None = None) -> dict:
    """Assert that the FP64 oracle certifies a GPU result `out` (a Solver.solve() or
    solve_packed() dict) of `solver` on `prob` to relative gap and infeasibility <= tol.
    Returns the oracle's figures."""
    prm = solver.params
    sigma, _ = solver.scaling()
    y_s = np.asarray(out["y"], dtype=np.float64) / sigma
    pr = solver.primal()
    st = solver.step_iterate(0, prm.k_c + prm.k_p)
    # A X_{t+1}, <C_s, X_{t+1}> rebuilt by the oracle from the tracked state
    AX, cX = orc.primal_from_model_update(prob, st["zbar"], st["cbar"], pr["V"], pr["S"], prm.alpha, prm.k_p)
    scale = 1.0 + np.abs(AX).max()
    assert np.abs(pr["AX"] - AX).max() <= 1e-9 * scale, np.abs(pr["AX"] - AX).max()
    # <C, X> goes through the library's products with C: FP32 accumulation for FP32 / BF16
    # values (unit round-off 6e-8, a few hundred terms per entry of V^T C V)
    c_tol = 1e-9 if prm.precision == "f64" else 2e-6
    assert abs(pr["cX"] - cX) <= c_tol * (1 + abs(cX)), (pr["cX"], cX)
    assert abs(pr["cX"] - out["primal_obj_scaled"]) <= 1e-12 * (1 + abs(cX))
    lam_max = None
    if lanczos_steps is not None:
        lam_max = orc.lambda_max_sparse(prob, orc.proj_Y(prob, y_s), steps=lanczos_steps)
    cert = orc.certificate(prob, y_s, AX, cX, alpha=prm.alpha, units=units, dense=dense, lam_max=lam_max)
    say(f"oracle certificate: f {cert['f']:.10e} (gpu {out['f_scaled']:.10e}) gap {cert['rel_gap']:.3e} "
        f"infeas {cert['rel_infeas']:.3e} (gpu {out['rel_gap']:.3e} / {out['rel_infeas']:.3e})")
    assert abs(cert["f"] - out["f_scaled"]) <= f_tol * (1 + abs(cert["f"])), (cert["f"], out["f_scaled"])
    assert cert["rel_gap"] <= tol + 1e-9, cert
    assert cert["rel_infeas"] <= tol + 1e-9, cert
    if check_sketch and out.get("U") is not None and out.get("lam") is not None:
        # the library evaluates <C, Xhat> with its product precision, A(Xhat) always in FP64
        c_tol = 1e-8 if prm.precision == "f64" else 2e-6
        cx_hat, inf_hat = orc.sketch_certificate(prob, out["U"], out["lam"], units)
        say(f"sketch: <C, Xhat> {cx_hat:.10e} (gpu {out['sketch_primal_obj']:.10e}) infeas {inf_hat:.3e} "
            f"(gpu {out['sketch_rel_infeas']:.3e})")
        assert abs(cx_hat - out["sketch_primal_obj"]) <= c_tol * (1 + abs(cx_hat)), (cx_hat, out["sketch_primal_obj"])
        assert abs(inf_hat - out["sketch_rel_infeas"]) <= 1e-8 * (1 + inf_hat), (inf_hat, out["sketch_rel_infeas"])
        cert["sketch_primal_obj"] = cx_hat
        cert["sketch_rel_infeas"] = inf_hat
    cert["AX"] = AX
    cert["cX"] = cX
    return cert
