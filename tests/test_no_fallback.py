"""The product path has no CPU fallback: without the built library the binding refuses to
import, and without a GPU the library refuses to create a context (no silent host path)."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_binding_refuses_to_import_without_the_library(tmp_path):
    pkg = tmp_path / "paper_2312_05837_amd"
    pkg.mkdir()
    shutil.copy(os.path.join(ROOT, "paper_2312_05837_amd", "__init__.py"), pkg / "__init__.py")
    r = subprocess.run([sys.executable, "-c", "import paper_2312_05837_amd"], cwd=tmp_path, capture_output=True,
                       text=True, timeout=300)
    assert r.returncode != 0
    assert "ImportError" in r.stderr and "no CPU fallback" in r.stderr


def test_no_context_without_a_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present: contexts are created there")
    sys.path.insert(0, ROOT)
    import paper_2312_05837_amd as P
    with pytest.raises(P.IsingError) as e:
        P.ising_create(0)
    assert e.value.status in (P.ISING_EDEVICE, P.ISING_EINVAL)
