"""The C-ABI library loads on a machine without a GPU and exports every function include/vx.h
declares; host-side paths that need no device behave as documented."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "vx.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^[A-Za-z_][\w \*]*?\b(vx_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_api():
    names = declared_functions()
    for n in ("vx_create", "vx_destroy", "vx_winding", "vx_refine", "vx_gen_tangle", "vx_gen_line_ring"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_1911_12070_amd as vx
    lib = vx.lib()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(declared_functions()) <= set(vx.EXPORTS)


def test_network_size_constants_agree():
    """The surrogate's sizes in the header, the binding, the seeded initial weights and the committed
    weights file describe one network: 128 inputs, hidden width H, 4 outputs."""
    import numpy as np

    import paper_1911_12070_amd as vx
    import vxinputs
    text = open(os.path.join(ROOT, "include", "vx.h")).read()
    c = {k: int(v) for k, v in re.findall(r"#define VX_MLP_(NIN|NHID|NOUT|NPARAMS) (\d+)", text)}
    nin, h, nout = c["NIN"], c["NHID"], c["NOUT"]
    assert c["NPARAMS"] == nin * h + h + h * h + h + h * nout + nout
    assert vx.MLP_NHID == h and vx.MLP_NPARAMS == c["NPARAMS"]
    assert vxinputs.MLP_NHID == h and vxinputs.MLP_NPARAMS == c["NPARAMS"]
    assert vxinputs.mlp_pack(vxinputs.mlp_init(0)).size == c["NPARAMS"]
    path = os.path.join(ROOT, "paper_1911_12070_amd", "weights", "surrogate_c2.bin")
    raw = open(path, "rb").read()
    assert raw[:6] == b"VXMLP1"
    assert int(np.frombuffer(raw[8:16], np.int64)[0]) == c["NPARAMS"] and len(raw) == 16 + 4 * c["NPARAMS"]
    w = np.frombuffer(raw[16:], np.float32)
    assert np.isfinite(w).all() and np.abs(w).max() > 0


def test_status_strings_and_defaults():
    import paper_1911_12070_amd as vx
    lib = vx.lib()
    assert lib.vx_status_str(0) == b"VX_OK"
    assert lib.vx_status_str(-2) == b"VX_ERR_CAPACITY"
    assert vx.vx_version() >= 10000
    p = vx.vx_refine_defaults()
    assert p.max_descent == 32 and p.max_newton == 20 and abs(p.newton_tol - 1e-6) < 1e-12


def test_null_handle_is_rejected():
    import paper_1911_12070_amd as vx
    lib = vx.lib()
    assert lib.vx_wind_config(None, 0) == vx.VX_ERR_INVALID
    assert lib.vx_profile_enable(None, 1) == vx.VX_ERR_INVALID
    assert lib.vx_destroy(None) == vx.VX_OK
    d = vx.dims(8, 8, 8)
    assert lib.vx_winding(None, d, None, None, None) == vx.VX_ERR_INVALID
    assert lib.vx_last_error(None) == b""


def test_create_without_gpu_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    import paper_1911_12070_amd as vx
    h = ctypes.c_void_p()
    st = vx.lib().vx_create(0, ctypes.byref(h))
    assert st != vx.VX_OK and not h.value


def test_product_package_does_not_reach_the_oracle():
    pkg = os.path.join(ROOT, "paper_1911_12070_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text.replace("Oracle", "").lower().replace("oracle-free", ""), f
