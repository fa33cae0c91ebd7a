"""GPU: the handle-free sketch update that allocates no device memory
(usbs_sketch_update_noalloc) against the handle entry point usbs_op_sketch_update,
through the C ABI, on two calls in a row (the second smaller than the first)."""
import numpy as np
import pytest

import sdp_inputs as si

pytestmark = pytest.mark.gpu


def test_noalloc_sketch_update_equals_handle_entry_point(cuda):
    import torch
    from paper_2312_11801_amd import Params, Solver, UsbsError
    from paper_2312_11801_amd.native import sketch_update_noalloc
    rng = np.random.default_rng(21)
    stream = torch.cuda.current_stream().cuda_stream
    for n, q, g in ((3001, 11, 0.37), (517, 5, 0.0)):
        print(f"noalloc sketch update: n={n} q={q} g={g}", flush=True)
        prob = si.maxcut_er(n, 6.0 / n, seed=n)
        psi = si.test_matrix(n, 10, seed=n)
        s = Solver(prob, Params(k_c=3, k_p=0, lanczos_max_restarts=2), psi=psi)
        W = torch.tensor(rng.standard_normal((n, q)), dtype=torch.float64, device="cuda")
        lam = rng.random(q) + 0.1
        P0 = torch.tensor(rng.standard_normal((n, 10)), dtype=torch.float64, device="cuda")
        P_ref = P0.clone()
        s.op_sketch_update(g, W, lam, P_ref)
        psi_dev = torch.tensor(psi, dtype=torch.float32, device="cuda")
        P_new = P0.clone()
        sketch_update_noalloc(g, W, lam, psi_dev, P_new, stream)
        torch.cuda.synchronize()
        s.free()
        a, b = P_new.cpu().numpy(), P_ref.cpu().numpy()
        # the same kernels in the same order: bit for bit
        assert np.array_equal(a, b), np.abs(a - b).max()
        # and the Sec. 4 update itself, in FP64 on the host
        Wn = W.cpu().numpy()
        ref = g * P0.cpu().numpy() + (Wn * lam[None, :]) @ (Wn.T @ psi.astype(np.float64))
        assert np.abs(a - ref).max() <= 1e-11 * (1 + np.abs(ref).max())
    # sizes beyond the maximum are refused with a message, before any launch
    W = torch.zeros((8, 17), dtype=torch.float64, device="cuda")
    with pytest.raises(UsbsError, match="q and r must be in"):
        sketch_update_noalloc(1.0, W, np.ones(17), torch.zeros((8, 10), dtype=torch.float32, device="cuda"),
                              torch.zeros((8, 10), dtype=torch.float64, device="cuda"), stream)
