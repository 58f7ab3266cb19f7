"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Builds the oracle (oracle/oracle.c), the library's host code
(paper_1805_06019_amd/csrc/host.cpp: encoder, stream validator, decoder
initialisation with the block directory and the strip-table builders) and
tests/sanitize_driver.cpp with -fsanitize=address,undefined, then runs the
driver: ten geometries (block sizes 2/4/8, tree heights 1-6, ragged images, a
restricted range mask) encoded by both encoders (streams compared byte for
byte), decoded and rendered by the oracle, validated and initialised by the
library, and 160 bit-flipped and 48 truncated copies of each stream through
the validator and the initialisation.  Any sanitizer report fails the test.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-g", "-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]
HIP_INC = ["-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"]


@pytest.mark.skipif(not shutil.which("g++") or not os.path.exists("/opt/rocm/lib/libamdhip64.so"),
                    reason="needs g++ and the HIP runtime library to link against")
def test_host_code_under_sanitizers(tmp_path):
    objs = {
        "oracle.o": ["gcc", "-std=c11", *SAN, "-c", os.path.join(ROOT, "oracle", "oracle.c")],
        "host.o": ["g++", "-std=c++17", *SAN, *HIP_INC, "-c",
                   os.path.join(ROOT, "paper_1805_06019_amd", "csrc", "host.cpp")],
        "driver.o": ["g++", "-std=c++17", *SAN, *HIP_INC, "-c", os.path.join(ROOT, "tests", "sanitize_driver.cpp")],
    }
    procs = []
    for name, cmd in objs.items():
        procs.append((name, subprocess.Popen(cmd + ["-o", str(tmp_path / name)], stdout=subprocess.PIPE,
                                             stderr=subprocess.STDOUT, text=True)))
    for name, p in procs:
        out, _ = p.communicate(timeout=600)
        assert p.returncode == 0, f"building {name}:\n{out}"
    exe = str(tmp_path / "sanitize_driver")
    subprocess.run(["g++", *SAN, *[str(tmp_path / n) for n in objs], "-L/opt/rocm/lib", "-lamdhip64",
                    "-lpthread", "-lm", "-o", exe], check=True, timeout=300)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1",
               HIP_VISIBLE_DEVICES="", OMP_NUM_THREADS="4")
    r = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, env=env, timeout=900)
    assert r.returncode == 0 and "ERROR: AddressSanitizer" not in r.stdout and "runtime error" not in r.stdout, \
        r.stdout[-6000:]
    assert "10 geometries, 0 failures" in r.stdout
