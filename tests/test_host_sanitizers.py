"""The library's host code under AddressSanitizer and UBSan (no GPU): the
operator builders of host_math.cpp swept over every supported size, spin,
order and cutoff, and the tuning-table parser of tuning.cpp fed a malformed
table.  Host-only builds (g++; hipcc with the sanitizer on the host side
only for the file that includes the HIP headers)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1104_3408_amd", "csrc")
INC = os.path.join(os.path.dirname(HERE), "include")
HIPCC = "/opt/rocm/bin/hipcc"
SAN = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all"]


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600, **kw)
    assert r.returncode == 0, (cmd[0], r.stdout[-2000:], r.stderr[-4000:])
    return r.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_math_under_sanitizers(tmp_path):
    exe = str(tmp_path / "sweep")
    _run(["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer"] + SAN +
         ["-I" + CSRC, os.path.join(HERE, "host", "host_math_sweep.cpp"), os.path.join(CSRC, "host_math.cpp"),
          "-o", exe])
    assert _run([exe]).startswith("ok")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="needs hipcc")
def test_tuning_parser_under_sanitizers(tmp_path):
    exe = str(tmp_path / "parse")
    host_san = []
    for f in SAN:
        host_san += ["-Xarch_host", f]
    _run([HIPCC, "--offload-arch=gfx950", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer"] + host_san +
         ["-I" + CSRC, "-I" + INC, os.path.join(HERE, "host", "tuning_table_parse.cpp"),
          os.path.join(CSRC, "tuning.cpp"), "-o", exe, "-ldl"])
    out = _run([exe, str(tmp_path / "table.txt")], env={**os.environ, "SG_TUNING_FILE": ""})
    assert out.strip().endswith("ok"), out
