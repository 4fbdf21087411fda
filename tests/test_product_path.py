"""The product path has no CPU fallback and does not use the oracle."""
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1810_02916_amd")


def test_missing_library_fails_loudly(tmp_path):
    """With libnf.so absent, the binding raises instead of computing anything."""
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "from paper_1810_02916_amd import _lib\n"
        "_lib.LIB_PATH = %r\n"
        "try:\n"
        "    _lib.load()\n"
        "except RuntimeError as e:\n"
        "    print('raised', 'missing' in str(e))\n"
        "else:\n"
        "    print('loaded')\n" % (ROOT, str(tmp_path / "libnf.so")))
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, check=True)
    assert out.stdout.strip() == "raised True"


def test_package_never_imports_the_oracle():
    for dirpath, _, files in os.walk(PKG):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle\b", text, re.M), f
                assert "nf_oracle" not in text and "liboracle" not in text, f
    for f in os.listdir(os.path.join(ROOT, "include")):
        assert "oracle" not in open(os.path.join(ROOT, "include", f)).read().lower(), f

