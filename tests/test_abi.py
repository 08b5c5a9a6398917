"""The C ABI: libsap.so loads without a GPU and exports every function that
include/sap.h declares; the binding names the same set.  No compute calls."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sap.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n.startswith(("sap_", "sps_"))))


@pytest.fixture(scope="module")
def libsap():
    import paper_2506_03070_amd as sap
    if not os.path.exists(sap.LIB_PATH):
        from paper_2506_03070_amd import build
        build.build()
    return ctypes.CDLL(sap.LIB_PATH)


def test_header_parses():
    names = declared_functions()
    for n in ["sap_create", "sap_destroy", "sps_generate", "sps_apply", "sap_qr", "sap_trsv", "sap_solve",
              "sap_lsqr"]:
        assert n in names


def test_every_declared_symbol_exported(libsap):
    missing = [n for n in declared_functions() if not hasattr(libsap, n)]
    assert not missing, missing


def test_binding_covers_header():
    import paper_2506_03070_amd as sap
    assert sorted(sap.EXPORTS) == declared_functions()


def test_status_strings(libsap):
    libsap.sap_status_string.restype = ctypes.c_char_p
    assert libsap.sap_status_string(0) == b"SAP_OK"
    assert libsap.sap_status_string(3) == b"SAP_RANK_DEFICIENT"


def test_null_arguments_rejected(libsap):
    """Argument checks run on the host before any device work."""
    assert libsap.sap_create(None, 0, 0) == 1          # SAP_EINVAL
    assert libsap.sps_generate(None, None, None) == 1
    assert libsap.sap_solve(None, None, None, None, None, None) == 1


def test_product_does_not_import_oracle():
    """The product package never reaches the CPU oracle."""
    pkg = os.path.join(ROOT, "paper_2506_03070_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "from oracle" not in src and "sap_oracle" not in src, f
