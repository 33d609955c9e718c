"""The C-ABI library loads on the host and exports every entry point the
public header declares; the binding's constants match the header."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "libkftrack.h")
LIB = os.path.join(ROOT, "paper_1711_06571_amd", "libkftrack.so")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(names))


def _defines():
    return {k: int(v) for k, v in re.findall(r"#define\s+(KF_[A-Z0-9_]+)\s+(\d+)", open(HEADER).read())}


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ["kf_seed", "kf_fit", "hit_bin", "kf_build", "hit_bin_workspace_bytes",
                     "kf_build_workspace_bytes", "kf_status_string", "kf_last_error"]:
        assert required in names, required


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.skip("libkftrack.so not built")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_constants_match_header():
    d = _defines()
    from paper_1711_06571_amd import kftrack
    assert kftrack.KF_OK == d["KF_OK"] and kftrack.KF_E_INVALID_ARG == d["KF_E_INVALID_ARG"]
    assert kftrack.KF_E_WORKSPACE == d["KF_E_WORKSPACE"] and kftrack.KF_E_HIP == d["KF_E_HIP"]
    assert kftrack.KF_E_UNSUPPORTED == d["KF_E_UNSUPPORTED"]
    for k in ["NO_CROSSING", "OUT_OF_Z", "NONFINITE", "S_NOT_PD", "CAP_TRUNC", "EVENT_TOO_LARGE"]:
        assert getattr(kftrack, "TRK_" + k) == d["KF_TRK_" + k]
    assert kftrack.LAYER_BARREL == d["KF_LAYER_BARREL"] and kftrack.LAYER_DISK == d["KF_LAYER_DISK"]
    assert kftrack.ARITH_F32 == d["KF_ARITH_F32"] and kftrack.ARITH_F64 == d["KF_ARITH_F64"]


def test_status_strings_on_host():
    if not os.path.exists(LIB):
        pytest.skip("libkftrack.so not built")
    lib = ctypes.CDLL(LIB)
    lib.kf_status_string.restype = ctypes.c_char_p
    assert lib.kf_status_string(0) == b"ok"
    assert lib.kf_status_string(1) == b"invalid argument"


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """Without the HIP library every entry point raises: there is no
    fallback implementation of any step."""
    from paper_1711_06571_amd import kftrack
    monkeypatch.setattr(kftrack, "LIB_PATH", str(tmp_path / "absent" / "libkftrack.so"))
    monkeypatch.setattr(kftrack, "_lib", None)
    with pytest.raises(kftrack.KFError, match="no fallback"):
        kftrack.lib()
    with pytest.raises(kftrack.KFError):
        kftrack.hit_bin_workspace_bytes(1, 17, 63, 16, 100)
