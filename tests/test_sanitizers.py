"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The C oracle and the host-only sources of the library (kpm_error.cpp,
kpm_lattice.cpp, kpm_transport.cpp) are built with gcc / g++
-fsanitize=address,undefined (every report fatal) and driven by
tests/sanitized_host.py in a child interpreter with the ASan runtime
preloaded.  The child must exit cleanly, and its results must equal those of
the ordinary builds (liborc.so, libkpm.so) on the same inputs."""
import json
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1307_0288_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1", "-fPIC", "-shared"]


def _runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = p.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.fixture(scope="module")
def builds(tmp_path_factory):
    if not shutil.which("gcc") or not shutil.which("g++") or not _runtime("libasan.so"):
        pytest.skip("gcc with the sanitizer runtimes is not available")
    d = tmp_path_factory.mktemp("san")
    orc = str(d / "liborc_san.so")
    host = str(d / "libkpm_host_san.so")
    subprocess.run(["gcc", "-std=c99"] + SAN + ["-o", orc, os.path.join(ROOT, "oracle", "kpm_oracle.c"),
                    "-lm"], check=True)
    subprocess.run(["g++", "-std=c++17"] + SAN +
                   ["-I", os.path.join(ROOT, "include"), "-I", CSRC, "-o", host] +
                   [os.path.join(CSRC, f) for f in ("kpm_error.cpp", "kpm_lattice.cpp",
                                                    "kpm_transport.cpp")], check=True)
    return orc, host


def test_host_code_is_clean_under_asan_and_ubsan(builds):
    orc, host = builds
    env = dict(os.environ)
    env["LD_PRELOAD"] = _runtime("libasan.so")
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:exitcode=86"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1:exitcode=87"
    p = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "sanitized_host.py"), orc, host],
                       capture_output=True, text=True, env=env, timeout=600)
    assert p.returncode == 0, p.stderr[-4000:]
    assert "runtime error" not in p.stderr and "AddressSanitizer" not in p.stderr, p.stderr[-4000:]
    got = json.loads(p.stdout.strip().splitlines()[-1])

    kp = pytest.importorskip("paper_1307_0288_amd")
    try:
        kp.lib()
    except ImportError:
        pytest.skip("libkpm.so is not built")
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import sanitized_host as sh
    import oracle.core as ocore
    saved = (ocore._LIB, sh.kb._lib)
    try:
        ref = sh.run(ocore._lib(), kp.lib())
    finally:
        ocore._LIB, sh.kb._lib = saved
    assert got.keys() == ref.keys()
    for k in ref:
        a, b = np.asarray(got[k]), np.asarray(ref[k])
        assert a.shape == b.shape, k
        assert np.allclose(a, b, rtol=1e-12, atol=1e-13, equal_nan=True), k
    assert got["invalid_range"] == [1.0] and got["invalid_asym"] == [1.0]
    assert got["invalid_nan"] == [1.0]
