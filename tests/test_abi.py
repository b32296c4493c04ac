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
    small = lbe.make_config(4, 32, 32, [12.0])  # periodic edge shorter than the range
    with pytest.raises(lbe.LBEError):
        lbe.workspace_bytes(small)
    assert b"kT" in L.lbe_last_error() or b"range" in L.lbe_last_error()
