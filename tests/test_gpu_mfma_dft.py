"""GPU: the measurement program that compares one 32-point DFT stage of the
line passes on the matrix cores (DFT-as-GEMM, v_mfma_f32_32x32x2f32) with the
register codelet.  Both must match a float64 direct DFT (forward then inverse
stage) to 1e-5 relative L2; the timing itself is reported by
`bench.py --workload mfma`, not asserted."""

import json
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

EXE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1510_04331_amd",
                   "dft32_mfma")


def test_mfma_and_codelet_stages_match_direct_dft():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    assert os.path.exists(EXE), "dft32_mfma is not built"
    print("dft32 mfma vs codelet", flush=True)
    r = subprocess.run([EXE, str(1 << 17), "8"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, (r.returncode, r.stdout, r.stderr)
    res = json.loads(r.stdout.strip().splitlines()[-1])
    assert res["valu_codelet"]["rel_l2_vs_direct_dft"] < 1e-5
    assert res["mfma_32x32x2_f32"]["rel_l2_vs_direct_dft"] < 1e-5
