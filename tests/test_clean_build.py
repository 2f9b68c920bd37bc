"""The committed tree builds from scratch: `build()` of __graft_entry__ on a
copy of HEAD with no built library compiles libtnlm.so (hipcc, gfx950) and
the oracle, after which the package imports and the library loads. Needs
hipcc and git, no GPU."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("git") is None
                    or not os.path.isdir(os.path.join(ROOT, ".git"))
                    or not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="needs git, a git checkout and hipcc")
def test_build_from_a_clean_checkout(tmp_path):
    dst = tmp_path / "src"
    dst.mkdir()
    arch = subprocess.run(["git", "-C", ROOT, "archive", "HEAD"],
                          capture_output=True, check=True).stdout
    subprocess.run(["tar", "-x", "-C", str(dst)], input=arch, check=True)
    lib = dst / "paper_1201_2450_amd" / "libtnlm.so"
    assert not lib.exists()
    # the package imports before anything is built; the library is only
    # loaded on first use
    r = subprocess.run([sys.executable, "-c", "import paper_1201_2450_amd"],
                       cwd=dst, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([sys.executable, "-c",
                        "import __graft_entry__ as g; g.build()"],
                       cwd=dst, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert lib.exists() and (dst / "oracle" / "libtnlm_oracle.so").exists()
    assert (dst / "oracle" / "libct_oracle.so").exists()
    assert "tnlm" in r.stdout
    r = subprocess.run([sys.executable, "-c",
                        "from paper_1201_2450_amd import _lib;"
                        "print(_lib.lib.tnlm_version().decode(),"
                        " len(_lib.header_functions()))"],
                       cwd=dst, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    assert r.stdout.startswith("tnlm")
