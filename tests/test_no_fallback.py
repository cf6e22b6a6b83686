"""The product path has no CPU fallback: without the built library every
entry point raises, and no module of the package imports the oracle."""

import ast
import subprocess
import sys
from pathlib import Path

ROOT = Path(__file__).resolve().parent.parent
PKG = ROOT / "paper_2104_10523_amd"


def test_missing_library_raises():
    code = (
        "import pathlib, sys\n"
        "import paper_2104_10523_amd as tn\n"
        "from paper_2104_10523_amd import _native\n"
        "_native._lib = None\n"
        "_native.LIB_PATH = pathlib.Path('/nonexistent/libtn.so')\n"
        "try:\n"
        "    tn.tn_build_network(2, [('h', [0])])\n"
        "except RuntimeError as e:\n"
        "    assert 'native library missing' in str(e), e\n"
        "    sys.exit(0)\n"
        "sys.exit(3)\n"
    )
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr


def test_package_never_imports_the_oracle():
    offenders = []
    for src in PKG.rglob("*.py"):
        tree = ast.parse(src.read_text())
        for node in ast.walk(tree):
            if isinstance(node, ast.Import):
                names = [a.name for a in node.names]
            elif isinstance(node, ast.ImportFrom):
                names = [node.module or ""]
            else:
                continue
            if any(n == "oracle" or n.startswith("oracle.") for n in names):
                offenders.append(f"{src.relative_to(ROOT)}:{node.lineno}")
    assert not offenders, offenders


def test_native_sources_never_reference_the_oracle():
    srcs = [p for p in (PKG / "csrc").iterdir() if p.suffix in (".hip", ".cpp", ".hpp", ".h")]
    srcs += list((ROOT / "include").glob("*.h"))
    assert srcs
    for src in srcs:
        assert "oracle" not in src.read_text().lower(), src
