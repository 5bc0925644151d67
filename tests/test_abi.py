"""Host-side checks of the C ABI: the library loads, exports every function
include/dse.h declares, and rejects invalid parameters before touching a GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dse.h")
LIB = os.path.join(ROOT, "paper_1206_1779_amd", "libdse.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dse_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    import torch  # noqa: F401  (binds the same HIP runtime the product uses)
    if not os.path.exists(LIB):
        import paper_1206_1779_amd.build as b
        b.build()
    from paper_1206_1779_amd import dse
    return dse.load()


def test_exports_every_declared_symbol(lib):
    names = declared()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_header():
    from paper_1206_1779_amd import dse
    assert sorted(dse.EXPORTS) == declared()


def test_defaults_and_sizes(lib):
    from paper_1206_1779_amd import dse
    p = dse.params()
    assert p.abi_version == 2 and p.n_z == 16 and abs(p.kappa - 0.5953525826) < 1e-9
    assert p.delta == -9 / 44 and p.gamma == -13 / 22
    n1 = lib.dse_workspace_bytes(C.byref(p))
    p2 = dse.params(n_z=64, n_g=64, n_rad=256, n_ir=64, n_ang=64)
    n2 = lib.dse_workspace_bytes(C.byref(p2))
    assert 0 < n1 < n2 < 64 << 20
    assert lib.dse_status_string(5) == b"Newton iteration did not converge"


@pytest.mark.parametrize("bad", [dict(n_z=0), dict(n_g=129), dict(eps2=-1.0), dict(lambda2=1e-9),
                                 dict(n_ang=0), dict(alpha_mu=0.0), dict(abi_version=7),
                                 dict(z_lambda_inv=0.0), dict(precision=5), dict(eps2=float("nan"))])
def test_invalid_params_rejected_before_launch(lib, bad):
    from paper_1206_1779_amd import dse
    p = dse.params(**bad)
    assert lib.dse_workspace_bytes(C.byref(p)) == 0
    h = C.c_void_p()
    st = lib.dse_init(C.byref(p), C.c_void_p(256), 1 << 30, None, C.byref(h))
    assert st == 1 and not h.value
    assert len(lib.dse_last_error(None)) > 0


def test_init_argument_checks(lib):
    from paper_1206_1779_amd import dse
    p = dse.params()
    h = C.c_void_p()
    assert lib.dse_init(C.byref(p), None, 1 << 30, None, C.byref(h)) == 1          # NULL workspace
    assert lib.dse_init(C.byref(p), C.c_void_p(1000), 1 << 30, None, C.byref(h)) == 1  # misaligned
    assert lib.dse_init(C.byref(p), C.c_void_p(256), 16, None, C.byref(h)) == 3    # too small
    assert lib.dse_residual(None, None, None, None) == 1
    assert lib.dse_destroy(None) == 0
