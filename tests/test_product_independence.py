"""The product package never imports the oracle (the oracle is test
infrastructure only): no source file under the package names it, and the
package and its training driver import with `oracle` made unimportable."""
from __future__ import annotations

import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1407_8315_amd")


def test_no_source_file_of_the_package_names_the_oracle():
    hits = []
    for dirpath, _, files in os.walk(PKG):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f), encoding="utf-8").read()
                if re.search(r"\boracle\b", text):
                    hits.append(os.path.relpath(os.path.join(dirpath, f), ROOT))
    assert hits == [], f"product sources mention the oracle: {hits}"


def test_package_and_training_driver_import_without_the_oracle():
    code = (
        "import sys\n"
        "sys.modules['oracle'] = None\n"          # any `import oracle` now raises ImportError
        "import paper_1407_8315_amd\n"
        "import runpy\n"
        "sys.argv = ['train_order_mlp', '--help']\n"
        "try:\n"
        "    runpy.run_module('paper_1407_8315_amd.train_order_mlp', run_name='__main__')\n"
        "except SystemExit as e:\n"
        "    assert e.code == 0, e.code\n"
        "assert 'oracle' not in [m for m in sys.modules if sys.modules[m] is not None]\n"
        "print('ok')\n"
    )
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip().endswith("ok")
