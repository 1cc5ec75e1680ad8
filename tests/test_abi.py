"""Host-side checks of the C-ABI library (no GPU needed)."""
import ctypes
import os
import re

import pytest

import paper_2203_06513_amd as ec

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ecpic.h")
HEADER2D = os.path.join(ROOT, "include", "ecpic2d.h")


def declared_symbols(header=HEADER, prefix="ecpic_"):
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(" + prefix + r"[a-z_0-9A-Z]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert declared_symbols() == sorted(ec.EXPORTS)
    assert declared_symbols(HEADER2D, "ecpic2d_") == sorted(ec.EXPORTS_2D)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(ec.LIB_PATH):
        pytest.fail("libecpic.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(ec.LIB_PATH)
    for name in declared_symbols() + declared_symbols(HEADER2D, "ecpic2d_"):
        assert hasattr(lib, name), name


def test_2d_invalid_config_without_device():
    """2D configurations outside the documented ranges are rejected before any
    device is touched."""
    bad = [dict(M1=12), dict(M2=4), dict(M1=1024), dict(degree=1), dict(degree=6), dict(dt=0.8),
           dict(tol=0.0), dict(n_particles=-1), dict(kmax=65), dict(L1=-1.0), dict(weight=float("nan")),
           dict(hbar=0.1), dict(spin=2), dict(spin=1, hbar=float("inf"))]
    for b in bad:
        args = dict(L1=8.0, L2=8.0, M1=16, M2=16, degree=3, n_particles=10, dt=0.05, tol=1e-12)
        args.update(b)
        with pytest.raises(ec.EcpicError) as e:
            ec.Context2D(**args)
        assert e.value.status == -1, b


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
