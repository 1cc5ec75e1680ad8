"""Host-side checks of the C-ABI library (no GPU needed)."""
import ctypes
import os
import re

import pytest

import paper_2203_06513_amd as ec

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ecpic.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ecpic_[a-z_0-9]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert declared_symbols() == sorted(ec.EXPORTS)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(ec.LIB_PATH):
        pytest.fail("libecpic.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(ec.LIB_PATH)
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_strerror_and_invalid_config_without_device():
    lib = ec.load()
    assert lib.ecpic_strerror(0) == b"ok"
    assert b"converge" in lib.ecpic_strerror(-3)
    # invalid configurations are rejected before any device is touched
    bad = [dict(degree=1), dict(degree=6), dict(M=4), dict(dt=1.0), dict(tol=0.0), dict(n_particles=-1),
           dict(waves_per_item=5), dict(splitting=2), dict(item_particles=3000), dict(item_particles=32768),
           dict(hbar=0.1), dict(spin=True, precision=1), dict(spin=True, warmstart=2),
           dict(spin=True, hbar=float("nan"))]
    for b in bad:
        args = dict(L=8.0, M=16, degree=3, n_particles=10, dt=0.05, tol=1e-12)
        args.update(b)
        with pytest.raises(ec.EcpicError) as e:
            ec.Context(**args)
        assert e.value.status == -1, b


def test_product_path_does_not_import_the_oracle():
    """The package and its sources never reference the CPU oracle."""
    pkg = os.path.join(ROOT, "paper_2203_06513_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text and "liboracle" not in text, f
