"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The oracle (plain C) is rebuilt with gcc's ASan and UBSan and the oracle
  pins run against it in a child process (the slow Boltzmann-relaxation pin
  aside): out-of-bounds accesses, use-after-free and undefined arithmetic in
  the oracle abort the child.
* The HIP library is rebuilt with ASan and UBSan on its host side only
  (device code is untouched; `-Xarch_host` keeps the sanitizers off the GPU
  compile) and the host-only ABI checks (exports, configuration validation,
  null handles, workspace sizes) run against it.

Both builds go to `_build_san/` directories (git-ignored) and are reused
while their sources do not change."""
import hashlib
import os
import shutil
import subprocess
import sys
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]
ORACLE_SRC = ROOT / "oracle" / "lbe_oracle.c"
CSRC = ROOT / "paper_1202_3842_amd" / "csrc"
SOURCES = ["lbe_kernels.hip", "lbe_api.hip", "lbe_adjoint.hip", "lbe_noalloc.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _digest(paths, flags):
    h = hashlib.sha256(" ".join(flags).encode())
    for p in paths:
        h.update(Path(p).read_bytes())
    return h.hexdigest()[:16]


def _gcc_runtime(name):
    out = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return out if out and Path(out).is_file() else None


def _clang_asan_runtime():
    for p in sorted(Path("/opt/rocm/llvm/lib/clang").glob("*/lib/linux/libclang_rt.asan-x86_64.so")):
        return str(p)
    return None


def _run_child(args, env_extra, timeout):
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env.setdefault("OMP_NUM_THREADS", "4")
    r = subprocess.run([sys.executable, *args], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=timeout)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
    return out


def test_oracle_pins_under_asan_and_ubsan(tmp_path):
    asan = _gcc_runtime("libasan.so")
    if shutil.which("gcc") is None or asan is None:
        pytest.skip("gcc with AddressSanitizer is not available")
    flags = ["-std=gnu11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=undefined", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC",
             "-shared"]
    out_dir = ROOT / "oracle" / "_build_san"
    out_dir.mkdir(exist_ok=True)
    lib = out_dir / f"liblbe_oracle_{_digest([ORACLE_SRC], flags)}.so"
    if not lib.exists():
        subprocess.run(["gcc", *flags, "-o", str(lib), str(ORACLE_SRC), "-lm"], check=True)
    env = {"LD_PRELOAD": asan, "LBEO_LIB": str(lib)}
    loaded = _run_child(["-c", "import oracle; oracle.lib(); print(oracle.LIB)"], env, 120)
    assert str(lib) in loaded
    _run_child(["-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
                "tests/test_oracle_tables.py", "tests/test_oracle_pins.py",
                "-k", "not relaxes_to_boltzmann"], env, 1500)


def test_abi_host_code_under_asan_and_ubsan():
    asan = _clang_asan_runtime()
    if not Path(HIPCC).exists() or asan is None:
        pytest.skip("hipcc with AddressSanitizer is not available")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-fno-omit-frame-pointer",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *san]
    srcs = [CSRC / s for s in SOURCES] + sorted(CSRC.glob("*.hpp")) + [ROOT / "include" / "lbe.h"]
    out_dir = ROOT / "paper_1202_3842_amd" / "_build_san"
    out_dir.mkdir(exist_ok=True)
    lib = out_dir / f"liblbe_{_digest(srcs, flags)}.so"
    if not lib.exists():
        objs = [out_dir / (Path(s).stem + ".o") for s in SOURCES]
        procs = [subprocess.Popen([HIPCC, *flags, "-I", str(ROOT / "include"), "-c", str(CSRC / s), "-o", str(o)],
                                  stderr=subprocess.DEVNULL) for s, o in zip(SOURCES, objs)]
        assert all(p.wait() == 0 for p in procs), "sanitizer build failed"
        subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *san, "-shared-libsan", "-o", str(lib),
                        *map(str, objs)], check=True)
    env = {"LD_PRELOAD": asan, "LBE_LIB": str(lib)}
    loaded = _run_child(["-c", "from paper_1202_3842_amd import lbe; lbe.lib(); print(lbe.LIB_PATH)"], env, 120)
    assert str(lib) in loaded
    _run_child(["-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "tests/test_abi.py"], env, 600)
