"""The C ABI used from plain C, with no Python or PyTorch in the process:
tests/c_example/solve_poisson.c assembles a 2-D Poisson system on the host,
copies it with the HIP runtime API and solves it with p-BiCGStab and residual
replacement (Algorithm 9 with Section 4.2's replacement)."""

import importlib.util
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(os.path.dirname(HERE), "paper_1612_01395_amd", "libpbcgs.so")


def _builder():
    spec = importlib.util.spec_from_file_location("c_example_build", os.path.join(HERE, "c_example", "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.skipif(not os.path.exists(LIB), reason="libpbcgs.so not built")
def test_c_example_compiles_and_reports_missing_device(tmp_path):
    """Compiles warning-free against include/pbcgs.h; without a GPU the context
    call returns an error (exit 2), it does not crash."""
    import torch
    exe = _builder().build(str(tmp_path / "solve_poisson"))
    if torch.cuda.is_available():
        pytest.skip("a GPU is present: the solve itself is the gpu test")
    res = subprocess.run([exe, "8"], capture_output=True, text=True, timeout=60)
    assert res.returncode == 2, (res.returncode, res.stdout, res.stderr)
    assert "no context" in res.stdout


@pytest.mark.gpu
@pytest.mark.parametrize("n", [16, 100])
def test_c_example_solves_on_gpu(n):
    """x = 1 recovered to 1e-8 from b = A 1 on an n x n Poisson grid."""
    b = _builder()
    exe = b.EXE if os.path.exists(b.EXE) else b.build()
    res = subprocess.run([exe, str(n)], capture_output=True, text=True, timeout=60)
    print(res.stdout, res.stderr)
    assert res.returncode == 0, (res.returncode, res.stdout, res.stderr)
    assert res.stdout.startswith("success after"), res.stdout
