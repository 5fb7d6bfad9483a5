"""The CPU tier under AddressSanitizer and UndefinedBehaviorSanitizer: the C
oracle and the host code of the HIP library are rebuilt with both
sanitizers (device code unchanged), and the `-m "not gpu"` tests run again
in a child process that preloads the sanitizer runtime and loads those
builds.  Any sanitizer report fails the child (halt on error), so this
test passes only on a clean run."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
IN_CHILD = os.environ.get("GCSS_SANITIZED") == "1"


@pytest.mark.skipif(IN_CHILD, reason="runs in the parent only")
def test_cpu_tier_is_clean_under_asan_and_ubsan(tmp_path):
    import oracle
    from paper_1312_6838_amd import build as libbuild
    rt = libbuild.asan_runtime()
    if not rt:
        pytest.skip("no clang AddressSanitizer runtime in the ROCm toolchain")
    orc = oracle.build_sanitized(str(tmp_path / "liboracle_asan.so"))
    lib = libbuild.build(out_dir=str(tmp_path), sanitize=True)
    env = dict(os.environ)
    env.update(LD_PRELOAD=rt, GCSS_SANITIZED="1", GCSS_LIBRARY=lib, GCSS_ORACLE_LIBRARY=orc,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "tests", "-x", "-q", "-m", "not gpu",
                        "-p", "no:cacheprovider"], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=1500)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert "passed" in out


@pytest.mark.skipif(not IN_CHILD, reason="checks the sanitized child process")
def test_child_loaded_the_sanitized_builds():
    import oracle
    from paper_1312_6838_amd import _abi
    _abi.load()
    oracle._load()
    maps = open("/proc/self/maps").read()
    assert os.environ["GCSS_LIBRARY"] in maps
    assert os.environ["GCSS_ORACLE_LIBRARY"] in maps
    assert "libclang_rt.asan" in maps
