"""Host-side helpers of the benchmark (no GPU)."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_source_hash_ignores_comments_only():
    """The stored counters are tied to the kernels' code: comments and layout
    may change without invalidating them, code and string literals may not."""
    sys.path.insert(0, ROOT)
    import bench
    base = "int f(int a) { return a + 1; } // note\nconst char *s = \"//x /*y*/\";\n"
    same = "/* new */ int f(int a)   {\n  return a + 1;   // other note\n}\nconst char *s = \"//x /*y*/\";\n"
    code = "int f(int a) { return a + 2; }\nconst char *s = \"//x /*y*/\";\n"
    lit = "int f(int a) { return a + 1; }\nconst char *s = \"//x /*z*/\";\n"
    t = bench._code_tokens
    assert t(base) == t(same)
    assert t(base) != t(code)
    assert t(base) != t(lit)
    assert "'/'" in t("char c = '/'; // c")
