"""The library's device reciprocal (recip_1_4, used by the sampling rule's
projection) equals the correctly rounded binary32 division for every input in
[1, 4), checked exhaustively on the GPU by tests/recip_check.hip (built by
__graft_entry__.build())."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "recip_check")


def test_reciprocal_is_correctly_rounded_on_1_4():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    assert os.path.exists(EXE), "tests/recip_check not built: run __graft_entry__.build()"
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "16777216 values in [1, 4): 0 mismatches" in r.stdout, r.stdout
