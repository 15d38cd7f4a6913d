"""Host-side checks of the C-ABI library (no GPU needed): it loads, and it
exports every function that include/fr_dvm.h declares."""
import ctypes
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_header_symbol():
    from paper_2312_06567_amd import frdvm
    if not os.path.exists(frdvm.LIB_PATH):
        pytest.fail("libfrdvm.so is not built (run __graft_entry__.build())")
    L = frdvm.lib()
    names = frdvm.header_functions()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_default_params_without_gpu():
    from paper_2312_06567_amd import frdvm
    p = frdvm._Params()
    frdvm.lib().fr_dvm_default_params(ctypes.byref(p))
    assert p.model == frdvm.BGK and p.precision == frdvm.FP64
    assert p.newton_tol == 1e-13 and p.newton_max_iter == 50 and p.omega == 0.81


def test_oracle_and_library_share_no_code():
    """The oracle neither imports the HIP package nor includes its sources."""
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    for fn in os.listdir(os.path.join(root, "oracle")):
        if fn.endswith((".py", ".c", ".h")):
            txt = open(os.path.join(root, "oracle", fn)).read()
            assert "import paper_2312_06567_amd" not in txt
            assert "from paper_2312_06567_amd" not in txt
            assert "frdvm_common" not in txt and "fr_dvm.h" not in txt


def test_mlp_input_width_agrees_everywhere():
    """FR_MLP_INPUTS of the header, the binding constant, the library's
    parameter count and the oracle network describe the same network."""
    import re
    from oracle import mlp as omlp
    from paper_2312_06567_amd import frdvm
    hdr = open(os.path.join(ROOT, "include", "fr_dvm_mlp.h")).read()
    n_in = int(re.search(r"#define FR_MLP_INPUTS (\d+)", hdr).group(1))
    assert n_in == frdvm.MLP_INPUTS == omlp.N_IN
    assert frdvm.lib().fr_mlp_param_count(64) == omlp.n_params(64)
