"""The C ABI library loads and exports every symbol include/usbs.h declares (no GPU calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "usbs.h")).read()
    return sorted(set(re.findall(r"\b(usbs_[a-z_A]+)\s*\(", src)))


def test_header_matches_binding_list():
    from paper_2312_11801_amd.native import EXPORTS
    assert sorted(EXPORTS) == _declared()


def test_library_exports_all_symbols():
    from paper_2312_11801_amd.native import LIB_PATH
    if not os.path.exists(LIB_PATH):
        pytest.skip("libusbs.so not built")
    lib = ctypes.CDLL(LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name


def test_struct_layout_matches_header():
    """Field order/types of the ctypes mirrors against the C structs (by parsing the header)."""
    from paper_2312_11801_amd import native
    src = open(os.path.join(ROOT, "include", "usbs.h")).read()
    for cname, py in (("usbs_problem", native.UsbsProblem), ("usbs_params", native.UsbsParams),
                      ("usbs_result", native.UsbsResult), ("usbs_server_config", native.UsbsServerConfig),
                      ("usbs_served_result", native.UsbsServedResult),
                      ("usbs_server_stats", native.UsbsServerStats)):
        body = re.search(r"typedef struct %s \{(.*?)\} %s;" % (cname, cname), src, re.S).group(1)
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        names = []
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            parts = decl.replace("*", " ").split()
            rest = " ".join(parts[1:]) if parts[0] != "const" else " ".join(parts[2:])
            names += [x.strip() for x in rest.split(",")]
        assert names == [f for f, _ in py._fields_], (cname, names)


def test_default_params_call_is_host_only():
    """usbs_default_params touches no device state and fills the App. E.1 defaults."""
    from paper_2312_11801_amd.native import LIB_PATH, UsbsParams, load_library
    if not os.path.exists(LIB_PATH):
        pytest.skip("libusbs.so not built")
    lib = load_library()
    p = UsbsParams()
    assert lib.usbs_default_params(ctypes.byref(p)) == 0
    assert (p.alpha, p.rho, p.beta, p.k_c, p.k_p, p.r) == (2.0, 0.01, 0.25, 10, 1, 10)


def test_footprint_is_host_only_and_monotone():
    """usbs_footprint_bytes (the server's admission estimate) is a host computation that
    grows with n and covers the n x 80 FP64 Lanczos basis."""
    from paper_2312_11801_amd.native import LIB_PATH, footprint_bytes, Params
    import sdp_inputs as si
    if not os.path.exists(LIB_PATH):
        pytest.skip("libusbs.so not built")
    a = footprint_bytes(si.maxcut_er(500, 0.02, seed=0), Params())
    b = footprint_bytes(si.maxcut_er(2000, 0.005, seed=0), Params())
    assert 0 < a < b
    assert b > 2000 * 80 * 8


def test_missing_library_raises(tmp_path):
    """No CPU fallback: loading from a path without the built library raises."""
    from paper_2312_11801_amd import native
    saved = native._LIB
    native._LIB = None
    try:
        with pytest.raises(FileNotFoundError):
            native.load_library(str(tmp_path / "libusbs.so"))
    finally:
        native._LIB = saved


def test_bench_refuses_several_gpus():
    """bench.py measures one GPU: --gpus 2 exits with status 2 and a message, touching no GPU."""
    import json
    import subprocess
    import sys
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert out.returncode == 2
    assert "one GPU" in json.loads(out.stdout.strip().splitlines()[-1])["error"]


def test_packed_structs_fit_the_launch_tables():
    """The packed kernel's per-instance state mirrors the header's phase count (usbs_packed_profile)."""
    src = open(os.path.join(ROOT, "include", "usbs.h")).read()
    ph = int(re.search(r"#define USBS_PACK_PHASES (\d+)", src).group(1))
    hdr = open(os.path.join(ROOT, "paper_2312_11801_amd", "csrc", "packed.h")).read()
    body = re.search(r"enum PackPhase \{(.*?)\};", hdr, re.S).group(1)
    names = [x.split("=")[0].split("//")[0].strip() for x in body.split("\n")]
    names = [x.rstrip(",") for x in names if x and not x.startswith("//")]
    assert names[-1] == "kPackPhases" and len(names) - 1 == ph
    from paper_2312_11801_amd.native import PACK_PHASES
    assert len(PACK_PHASES) == ph


@pytest.mark.parametrize("field,value,text", [
    ("k_c", 0, "k_c >= 1"), ("k_p", 12, "k_c + k_p"), ("r", 17, "0 <= r <= 16"),
    ("lanczos_steps", 9, "lanczos_steps"), ("rho", 0.0, "rho > 0"), ("beta", 1.0, "beta < 1"),
    ("lanczos_tol", 0.0, "tolerances"), ("autotune", 3, "autotune"), ("lanczos_max_restarts", -1, "restarts")])
def test_invalid_params_rejected_on_the_host(field, value, text):
    """usbs_create checks the parameters before it touches the device: each malformed field
    gives USBS_E_INVALID with a message that names it (header: error codes)."""
    from paper_2312_11801_amd.native import LIB_PATH, USBS_E_INVALID, Params, Solver, UsbsError
    import sdp_inputs as si
    if not os.path.exists(LIB_PATH):
        pytest.skip("libusbs.so not built")
    prm = Params()
    setattr(prm, field, value)
    with pytest.raises(UsbsError) as ei:
        Solver(si.maxcut_er(60, 0.1, seed=0), prm)
    assert ei.value.code == USBS_E_INVALID and text in str(ei.value), str(ei.value)


def test_noalloc_rejects_bad_sizes_on_the_host():
    """usbs_sketch_update_noalloc rejects sizes beyond its fixed scratch and NULL arguments
    with USBS_E_INVALID before any device call; the thread's message is read with
    usbs_last_error(NULL).  n = 0 is a no-op."""
    from paper_2312_11801_amd.native import LIB_PATH, USBS_E_INVALID, USBS_OK, load_library
    if not os.path.exists(LIB_PATH):
        pytest.skip("libusbs.so not built")
    lib = load_library()
    lam = (ctypes.c_double * 16)(*([1.0] * 16))
    fake = ctypes.c_void_p(16)   # never dereferenced: every case fails its host checks
    for n, q, r, ptr, text in ((100, 17, 10, fake, "q and r"), (100, 0, 10, fake, "q and r"),
                               (100, 4, 17, fake, "q and r"), (100, 4, 0, fake, "q and r"),
                               (-1, 4, 10, fake, "n must be"), (100, 4, 10, None, "NULL")):
        rc = lib.usbs_sketch_update_noalloc(n, q, r, 1.0, ptr, lam, ptr, ptr, None)
        assert rc == USBS_E_INVALID, (n, q, r)
        assert text in lib.usbs_last_error(None).decode()
    assert lib.usbs_sketch_update_noalloc(0, 4, 10, 1.0, None, lam, None, None, None) == USBS_OK
