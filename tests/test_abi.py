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


def test_workspace_at_the_node_limit(L):
    """Node indices are 32-bit: 1290^3 < 2^31 nodes is sized without overflow
    (per node the same bytes as 64^3, to within the halos), 1291^3 is refused."""
    for prec in (lbe.LBE_FP64, lbe.LBE_FP32_POP):
        per_node = lbe.workspace_bytes(lbe.make_config(64, 64, 64, [6.0], prec=prec)) / 64 ** 3
        big = lbe.workspace_bytes(lbe.make_config(1290, 1290, 1290, [6.0], prec=prec))
        assert 0.9 < big / 1290 ** 3 / per_node < 1.0, (prec, big)
    with pytest.raises(lbe.LBEError):
        lbe.workspace_bytes(lbe.make_config(1291, 1291, 1291, [6.0]))
    assert b"2^31" in L.lbe_last_error()


def test_adjoint_workspace_and_scope(L):
    cfg = lbe.make_config(32, 32, 32, [4.0], flags=lbe.LBE_PI_CARRIED)
    n1 = L.lbe_adjoint_workspace_bytes(C.byref(cfg), 100, 10)
    n2 = L.lbe_adjoint_workspace_bytes(C.byref(cfg), 100, 50)
    pop = 2 * 19 * 32 ** 3 * 8
    # 11 checkpoints + 10 tape slots vs 3 checkpoints + 50 tape slots
    assert n1 >= 11 * pop and n2 > n1
    bad = lbe.make_config(32, 32, 32, [4.0], flags=lbe.LBE_PI_CARRIED)
    assert L.lbe_adjoint_workspace_bytes(C.byref(bad), 10, 0) == 0
    assert b"segment" in L.lbe_last_error()
    # FP32 storage: checkpoints and tape states at half size, the adjoint state in FP64
    f32 = lbe.make_config(32, 32, 32, [4.0], prec=lbe.LBE_FP32_POP, flags=lbe.LBE_PI_CARRIED)
    assert 0 < L.lbe_adjoint_workspace_bytes(C.byref(f32), 100, 10) < n1
    # C^visc adds the padded J~ field to every tape slot and its adjoint fields
    visc = lbe.make_config(32, 32, 32, [4.0], flags=lbe.LBE_VISC | lbe.LBE_PI_CARRIED)
    assert L.lbe_adjoint_workspace_bytes(C.byref(visc), 100, 10) > n1
    assert L.lbe_adjoint_workspace_bytes(C.byref(cfg), 0, 5) == 0


def test_null_handles_are_rejected_without_touching_the_device(L):
    """Every entry point that takes a context, batch or adjoint handle returns
    LBE_ERR_ARG for a null handle (and the destroy calls accept one) before
    any HIP call, so this runs on a machine with no GPU."""
    o3 = (C.c_int * 3)(1, 1, 1)
    g3 = (C.c_double * 3)(0.0, 0.0, 0.0)
    calls = {
        "lbe_set_solid": (None, None, 0), "lbe_set_potential": (None, None, 0),
        "lbe_set_body_force": (None, 0, g3), "lbe_init_density": (None, 0, None, 0),
        "lbe_step": (None, 1), "lbe_step_phase": (None, 0), "lbe_get_density": (None, 0, None, 0),
        "lbe_get_velocity": (None, 0, None, 0), "lbe_get_momentum": (None, 0, None, 0),
        "lbe_get_force": (None, 0, 0, None, 0), "lbe_get_populations": (None, 0, 0, None, 0),
        "lbe_set_populations": (None, 0, 0, None, 0), "lbe_get_divergence": (None, None, 0),
        "lbe_get_quasipressure": (None, 0, o3, 0, None, 0), "lbe_init_quasipressure": (None, o3, 0),
        "lbe_set_quasipressure_route": (None, o3, 0),
        "lbe_get_quasipressure_noalloc": (None, 0, o3, 0, None),
        "lbe_diagnostics": (None, None), "lbe_synchronize": (None,),
        "lbe_set_force_zchunk": (None, 1), "lbe_set_force_tiling": (None, 1, 0, 0),
        "lbe_batch_step": (None, 1, 2), "lbe_adjoint_forward": (None,),
        "lbe_adjoint_backward": (None, None, None, None, 0, None, 0),
        "lbe_adjoint_state_grad": (None, 0, 0, None, 0),
        "lbe_adjoint_probe": (None, 0, 0, None, None),
        "lbe_adjoint_create": (None, 10, 5, None, 0, C.byref(C.c_void_p())),
        "lbe_create": (None, None, 0, None, C.byref(C.c_void_p())),
    }
    for name, args in calls.items():
        assert getattr(L, name)(*args) == lbe.LBE_ERR_ARG, name
    assert L.lbe_batch_box(None, 0) is None
    L.lbe_destroy(None)
    L.lbe_batch_destroy(None)
    L.lbe_adjoint_destroy(None)
    covered = set(calls) | {"lbe_batch_box", "lbe_destroy", "lbe_batch_destroy", "lbe_adjoint_destroy",
                            "lbe_workspace_bytes", "lbe_batch_workspace_bytes",
                            "lbe_adjoint_workspace_bytes", "lbe_last_error", "lbe_batch_create"}
    assert not set(lbe.declared_symbols()) - covered, set(lbe.declared_symbols()) - covered


def test_attraction_configuration_is_validated(L):
    """The attractive tail's parameters (lbe_config.att_eps, att_rc): the
    interaction range grows with att_rc, and bad values are refused before
    any device work."""
    base = lbe.workspace_bytes(lbe.make_config(32, 32, 32, [4.0]))
    with_att = lbe.workspace_bytes(lbe.make_config(32, 32, 32, [4.0], att_eps=0.2, att_rc=8.0))
    assert with_att > base                     # wider ghost layers of the fields
    bad = [
        (lbe.make_config(16, 16, 16, [2.0, 3.0], att_eps=[[0.1, 0.2], [0.1, 0.1]], att_rc=5.0), b"symmetric"),
        (lbe.make_config(16, 16, 16, [2.0], att_eps=-0.1, att_rc=5.0), b"symmetric"),
        (lbe.make_config(16, 16, 16, [4.0], att_eps=0.1, att_rc=4.0), b"att_rc"),
        (lbe.make_config(32, 32, 32, [4.0], att_eps=0.1, att_rc=9.5), b"att_rc"),
        (lbe.make_config(16, 16, 16, [2.0], att_eps=0.1, att_rc=5.0, flags=lbe.LBE_IDEAL), b"IDEAL"),
    ]
    for cfg, word in bad:
        with pytest.raises(lbe.LBEError):
            lbe.workspace_bytes(cfg)
        assert word in L.lbe_last_error(), L.lbe_last_error()
    ok = lbe.make_config(16, 16, 16, [2.0], att_eps=0.1, att_rc=5.0, flags=lbe.LBE_PI_CARRIED)
    assert L.lbe_adjoint_workspace_bytes(C.byref(ok), 10, 5) > 0      # the adjoint covers it
    arr = (lbe.lbe_config * 1)(ok)
    assert L.lbe_batch_workspace_bytes(arr, 1) > 0              # batches take it
    # ... but a batched box with it needs a hard-sphere shell to add to
    thin = (lbe.lbe_config * 1)(lbe.make_config(16, 16, 16, [0.4], att_eps=0.1, att_rc=3.0, flags=0))
    assert L.lbe_batch_workspace_bytes(thin, 1) == 0
    assert b"hard-sphere shell" in L.lbe_last_error()
