"""GPU: the request loop (usbs_server_*) with continuous batching.

Each request is a MaxCut SDP from the served-batch generator plus its grown version
(+1% vertices, warm-started from the resident state, Sec. 5.1).  The same requests are
served alone (one slot, one request at a time) and in a mix (several slots, extra
requests in flight, arrivals while others run); every result must be identical, and the
server's own solve must equal a direct usbs_create/usbs_solve/usbs_warm_start run.
"""
import numpy as np
import pytest

import sdp_inputs as si

pytestmark = pytest.mark.gpu

FIELDS = ("primal_obj", "dual_bound", "rel_gap", "rel_infeas", "iters", "descents", "status",
          "rel_gap_original", "lanczos_matvecs")


def _params():
    from paper_2312_11801_amd import Params
    # no time limit: the iteration count, hence every result, is independent of timing
    return Params(precision="f32", max_iters=150, time_limit=0.0)


def _requests(count, seed):
    reqs = si.served_batch(count=count, n_lo=300, n_hi=700, avg_degree=8.0, seed=seed)
    for q in reqs:
        q["psi"] = si.test_matrix(q["problem"].n, 10, seed=q["id"])
        q["psi_grown"] = si.test_matrix(q["grown"].n, 10, seed=q["id"])
    return reqs


def _key(res):
    return tuple(res[f] for f in FIELDS)


def test_served_alone_equals_mix_and_direct(cuda):
    from paper_2312_11801_amd import Server, Solver
    reqs = _requests(3, seed=3)
    fillers = _requests(2, seed=4)
    prm = _params()

    # alone: one slot, one request in the system at a time
    alone = {}
    sv = Server(slots=1, params=prm)
    for q in reqs:
        rid = sv.submit(q["problem"], q["psi"], q["grown"], q["psi_grown"])
        out = sv.wait(rid)
        alone[q["id"]] = (_key(out["base"]), _key(out["grown"]))
    sv.close()

    # mix: four slots, the requests interleaved with fillers, all submitted at once
    sv = Server(slots=4, params=prm)
    ids = {}
    for a, b in zip(reqs, fillers):
        ids[a["id"]] = sv.submit(a["problem"], a["psi"], a["grown"], a["psi_grown"])
        sv.submit(b["problem"], b["psi"], b["grown"], b["psi_grown"])
    ids[reqs[-1]["id"]] = sv.submit(reqs[-1]["problem"], reqs[-1]["psi"], reqs[-1]["grown"],
                                    reqs[-1]["psi_grown"])
    mixed = {k: sv.wait(v) for k, v in ids.items()}
    st = sv.stats()
    sv.close()
    assert st["peak_running"] >= 2, st
    for q in reqs:
        out = mixed[q["id"]]
        assert (_key(out["base"]), _key(out["grown"])) == alone[q["id"]], q["id"]
        assert out["t_submit"] <= out["t_admit"] <= out["t_base_done"] <= out["t_done"]

    # the server's solve is the library's solve
    q = reqs[0]
    s = Solver(q["problem"], prm, psi=q["psi"])
    base = s.solve(want_y=False)
    s.warm_start(q["grown"], psi=q["psi_grown"])
    grown = s.solve(want_y=False)
    s.free()
    b0, g0 = alone[q["id"]]
    assert tuple(base[f] for f in FIELDS) == b0
    assert tuple(grown[f] for f in FIELDS) == g0


def test_server_admission_by_footprint(cuda):
    """With a budget that fits only one request at a time, requests still all complete and
    never run together; a request larger than the whole budget is refused."""
    from paper_2312_11801_amd import Server, UsbsError, footprint_bytes
    reqs = _requests(3, seed=5)
    prm = _params()
    fps = [max(footprint_bytes(q["problem"], prm, q["psi"]), footprint_bytes(q["grown"], prm, q["psi_grown"]))
           for q in reqs]
    budget = int(max(fps) * 1.5)
    sv = Server(slots=3, params=prm, hbm_budget_bytes=budget)
    rids = [sv.submit(q["problem"], q["psi"], q["grown"], q["psi_grown"]) for q in reqs]
    outs = [sv.wait(r) for r in rids]
    st = sv.stats()
    assert st["peak_used_bytes"] <= budget and st["peak_running"] == 1, st
    big = si.maxcut_sparse_pm1(200000, 6.0, seed=1)
    with pytest.raises(UsbsError):
        sv.submit(big, si.test_matrix(big.n, 10, seed=0))
    sv.close()
    assert all(o["status_base"] >= 0 and o["status_grown"] >= 0 for o in outs)
