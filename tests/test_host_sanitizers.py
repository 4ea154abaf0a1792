"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer: the RE
compiler (paper_2503_06763_amd/csrc/compiler.cpp) and the request server's
arena (csrc/arena.hpp), built with g++ and run on the CPU
(tests/native/host_checks.cpp).  The REs: seeded random REs with and without
character sets, the fixed workload REs, malformed REs and random byte
strings."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from gen import regen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _res():
    out = [regen.to_re(regen.plain_small_re()), regen.to_re(regen.motif_re()), regen.to_re(regen.record_re()),
           regen.to_re(regen.csv_record_re()), regen.to_re(regen.csv_record_re(sets=True)),
           regen.to_re(regen.random_re(23))]
    for s in range(60):
        alpha = [b"ab", b"abcd", b"abcdefghijklmnopqrstuvwxyz", bytes(range(1, 128))][s % 4]
        try:
            out.append(regen.to_re(regen.random_re(9000 + s, n_ops=6 + s % 30, max_depth=4 + s % 5,
                                                   alphabet=alpha, set_p=0.4 if s % 2 else 0.0, max_tries=50)))
        except RuntimeError:
            pass
    out += [b"", b"(", b")", b"a)", b"(a", b"|", b"a|", b"|a", b"()", b"()*", b"a**", b"(a*)*", b"[", b"[]",
            b"[a", b"[z-a]", b"[^\\x00-\\xff]", b"\\", b"\\x4", b"\\xg0", b".*", b"(.|\\n)*", b"[a-c]+[^b]?",
            b"a" * 3000, b"(" * 200 + b"a" + b")" * 200, b"((((((((((a|b)*c)*d)*e)*f)*g)*h)*i)*j)*)"]
    rng = np.random.default_rng(4)
    for k in range(200):
        out.append(bytes(rng.choice(list(b"ab()|*+?[]^-.\\x01"), size=int(rng.integers(1, 24)))))
    return out


def test_compiler_and_arena_under_sanitizers(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "host_checks")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-I/opt/rocm/include", "-D__HIP_PLATFORM_AMD__", "-w",
           os.path.join(ROOT, "tests", "native", "host_checks.cpp"),
           os.path.join(ROOT, "paper_2503_06763_amd", "csrc", "compiler.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "sanitizer" in r.stderr.lower():
        pytest.skip("sanitizer runtime not available: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr[-4000:]
    res_file = tmp_path / "res.txt"
    res_file.write_text("\n".join(x.hex() for x in _res()) + "\n")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, str(res_file), "20000"], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0 and "runtime error" not in r.stderr and "ERROR:" not in r.stderr, \
        (r.stdout[-2000:], r.stderr[-4000:])
    assert r.stdout.strip().endswith("ok")
