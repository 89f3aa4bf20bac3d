"""The product path stands alone: the package imports nothing from oracle/
(the test-only FP64 reference) and its native sources include nothing from
there, and without the built HIP library every entry point raises instead of
computing anything on the host."""
import ast
import glob
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2108_13656_amd")


def test_package_imports_nothing_from_the_oracle():
    for fn in glob.glob(os.path.join(PKG, "**", "*.py"), recursive=True):
        tree = ast.parse(open(fn).read(), fn)
        for node in ast.walk(tree):
            if isinstance(node, ast.Import):
                names = [a.name for a in node.names]
            elif isinstance(node, ast.ImportFrom):
                names = [node.module or ""]
            else:
                continue
            assert not any(n == "oracle" or n.startswith("oracle.") for n in names), fn


def test_native_sources_include_nothing_from_the_oracle():
    for fn in glob.glob(os.path.join(PKG, "csrc", "*")) + glob.glob(os.path.join(ROOT, "include", "*")):
        for inc in re.findall(r'^\s*#\s*include\s*[<"]([^>"]+)[>"]', open(fn).read(), re.M):
            assert "oracle" not in inc and "decolor_ref" not in inc, (fn, inc)


def test_missing_library_raises():
    code = (
        "import paper_2108_13656_amd as P, torch\n"
        "P.LIB_PATH = '/nonexistent/libdecolor.so'\n"
        "P._lib = None\n"
        "for call in (lambda: P.lib(), lambda: P.validate([]),\n"
        "             lambda: P.decolorize(torch.zeros((2, 2, 3), dtype=torch.uint8))):\n"
        "    try:\n"
        "        call()\n"
        "    except (RuntimeError, TypeError) as e:\n"
        "        print('raised', type(e).__name__)\n"
        "    else:\n"
        "        print('returned')\n")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT,
                         timeout=300)
    assert out.returncode == 0, out.stderr
    lines = out.stdout.split()
    assert "returned" not in lines, out.stdout
    assert lines.count("raised") == 3, out.stdout
