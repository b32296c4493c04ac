"""Host-side checks of the C ABI library (no GPU needed): it loads, exports
every function include/lbe.h declares, and validates configurations."""
import ctypes as C
import subprocess

import pytest

from paper_1202_3842_amd import lbe


@pytest.fixture(scope="module")
def L():
    if not lbe.LIB_PATH.exists():
        from paper_1202_3842_amd import build
        build.build()
    return lbe.lib()


def test_every_declared_symbol_is_exported(L):
    declared = lbe.declared_symbols()
    assert "lbe_step" in declared and "lbe_create" in declared
    out = subprocess.run(["nm", "-D", "--defined-only", str(lbe.LIB_PATH)], check=True,
                         capture_output=True, text=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = [s for s in declared if s not in exported]
    assert not missing, missing
    for s in declared:
        getattr(L, s)


def test_workspace_size_and_validation(L):
    cfg = lbe.make_config(32, 32, 32, [4.0])
    n = lbe.workspace_bytes(cfg)
    # two ping-pong buffers of f~ and g~ (19 FP64 each) dominate
    assert n >= 2 * 2 * 19 * 32 ** 3 * 8
    cfg32 = lbe.make_config(32, 32, 32, [4.0], prec=lbe.LBE_FP32_POP)
    assert lbe.workspace_bytes(cfg32) < n
    bad = lbe.make_config(32, 32, 32, [4.0], kT=0.5)
    with pytest.raises(lbe.LBEError):
        lbe.workspace_bytes(bad)
    small = lbe.make_config(4, 32, 32, [6.0])  # periodic edge shorter than the range
    with pytest.raises(lbe.LBEError):
        lbe.workspace_bytes(small)
    assert b"range" in L.lbe_last_error()
    huge = lbe.make_config(32, 32, 32, [12.0])
    with pytest.raises(lbe.LBEError):
        lbe.workspace_bytes(huge)
    assert b"sigma" in L.lbe_last_error()


def test_adjoint_workspace_and_scope(L):
    cfg = lbe.make_config(32, 32, 32, [4.0], flags=0)
    n1 = L.lbe_adjoint_workspace_bytes(C.byref(cfg), 100, 10)
    n2 = L.lbe_adjoint_workspace_bytes(C.byref(cfg), 100, 50)
    pop = 2 * 19 * 32 ** 3 * 8
    # 11 checkpoints + 10 tape slots vs 3 checkpoints + 50 tape slots
    assert n1 >= 11 * pop and n2 > n1
    for bad in (lbe.make_config(32, 32, 32, [4.0], flags=lbe.LBE_VISC),
                lbe.make_config(32, 32, 32, [4.0], prec=lbe.LBE_FP32_POP, flags=0)):
        assert L.lbe_adjoint_workspace_bytes(C.byref(bad), 10, 5) == 0
    assert b"adjoint" in L.lbe_last_error()
    assert L.lbe_adjoint_workspace_bytes(C.byref(cfg), 0, 5) == 0
