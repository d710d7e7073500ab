"""The product path has no CPU fallback: with the HIP library missing, every
entry of the binding fails loudly (ImportError naming the build step), and the
package imports nothing from the oracle. CPU only."""
import ast
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1710_02261_amd")


def test_missing_library_fails_loudly():
    code = (
        "import paper_1710_02261_amd as ptk\n"
        "from paper_1710_02261_amd import _native\n"
        "_native._LIB_PATH = '/nonexistent/libptucker.so'\n"
        "_native._lib = None\n"
        "for call in (lambda: ptk.load_library(), lambda: ptk.Context((4, 4, 4), (2, 2, 2)),\n"
        "             lambda: ptk.fp64_rates(1), lambda: ptk.coo_scan('x', 3)):\n"
        "    try:\n"
        "        call()\n"
        "    except ImportError as e:\n"
        "        assert 'not built' in str(e), e\n"
        "    else:\n"
        "        raise SystemExit('no error')\n"
        "print('ok')\n")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                       cwd=ROOT, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.strip().endswith("ok")


def test_package_does_not_import_the_oracle():
    for name in os.listdir(PKG):
        if not name.endswith(".py"):
            continue
        tree = ast.parse(open(os.path.join(PKG, name)).read())
        for node in ast.walk(tree):
            if isinstance(node, ast.Import):
                mods = [a.name for a in node.names]
            elif isinstance(node, ast.ImportFrom):
                mods = [node.module or ""]
            else:
                continue
            assert not any(m == "oracle" or m.startswith("oracle.") for m in mods), name
