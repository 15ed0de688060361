"""The C-ABI library loads and exports every entry point include/soc.h
declares (no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "soc.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(soc_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("soc_build_grid", "soc_simulate_frequency", "soc_update_temperature", "soc_map",
                     "soc_trace_packages", "soc_ctx_create", "soc_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_1812_06632_amd", "libsoc.so"))
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_fails_loudly_without_library(tmp_path):
    """The Python binding has no CPU fallback: without libsoc.so it refuses
    to import."""
    import shutil
    import subprocess
    import sys
    pkg = tmp_path / "paper_1812_06632_amd"
    pkg.mkdir()
    shutil.copy(os.path.join(ROOT, "paper_1812_06632_amd", "soc.py"), pkg / "soc.py")
    (pkg / "__init__.py").write_text("")
    r = subprocess.run([sys.executable, "-c", "import paper_1812_06632_amd.soc"], cwd=str(tmp_path),
                       capture_output=True, text=True)
    assert r.returncode != 0 and "libsoc.so is missing" in r.stderr
