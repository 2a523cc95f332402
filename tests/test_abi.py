"""CPU checks of the C ABI boundary: the library loads, exports every function
include/pbcgs.h declares, reports errors without a GPU, and the product path
never touches the oracle."""

import ctypes
import os
import subprocess
import sys

import pytest

from paper_1612_01395_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_function():
    L = _lib.lib()
    names = _lib.declared_functions()
    assert len(names) >= 14
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    # the binding knows every declared function's signature
    assert set(names) <= set(_lib._SIGNATURES), set(names) - set(_lib._SIGNATURES)
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    assert set(names) <= exported


def test_status_strings_and_nnz_without_gpu():
    L = _lib.lib()
    for code, name in [(0, b"success"), (1, b"maxit"), (2, b"breakdown"), (3, b"nonfinite"),
                       (-1, b"invalid argument"), (-4, b"unsupported")]:
        assert L.pbcgs_status_str(code) == name
    import oracle
    for dim, npts in ((2, 5), (3, 7), (3, 27)):
        for n in (1, 2, 7, 64):
            assert L.pbcgs_convdiff_nnz(dim, n, npts) == oracle.assemble_nnz(dim, n, npts)
    assert L.pbcgs_convdiff_nnz(2, 8, 7) == _lib.ERR_INVALID_ARG


def test_null_arguments_are_rejected_not_crashing():
    L = _lib.lib()
    assert L.pbcgs_ctx_create(0, None, None) == _lib.ERR_INVALID_ARG
    assert L.pbcgs_ctx_destroy(None) == _lib.ERR_INVALID_ARG
    assert L.pbcgs_op_destroy(None) == _lib.ERR_INVALID_ARG
    assert L.pbcgs_op_rows(None) == _lib.ERR_INVALID_ARG
    assert L.pbcgs_op_index_bytes(None) == _lib.ERR_INVALID_ARG
    assert L.pbcgs_op_column_form(None) == _lib.ERR_INVALID_ARG
    assert _lib.last_error(None)


@pytest.mark.skipif(os.path.exists("/dev/kfd") and os.access("/dev/kfd", os.R_OK), reason="a GPU is present")
def test_context_creation_fails_cleanly_without_gpu():
    h = ctypes.c_void_p()
    rc = _lib.lib().pbcgs_ctx_create(0, None, ctypes.byref(h))
    assert rc < 0
    assert _lib.last_error(None)


def test_product_path_does_not_load_the_oracle():
    code = ("import sys; import paper_1612_01395_amd.solver, paper_1612_01395_amd._lib as L; L.lib(); "
            "print('oracle' in sys.modules)")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip() == "False"
    pkg = os.path.join(ROOT, "paper_1612_01395_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "liboracle" not in text, f


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; other counts exit with a message, before any GPU work."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_binding_constants_match_the_header():
    """Every PBCGS_ enumerator the header defines has the value the Python
    binding passes for it, and the binding's option maps cover them all."""
    import re
    from paper_1612_01395_amd import solver
    text = open(_lib.HEADER).read()
    enum = {m.group(1): int(m.group(2)) for m in re.finditer(r"\bPBCGS_([A-Z0-9_]+)\s*=\s*(-?\d+)", text)}
    for name in ("SUCCESS", "MAXIT", "BREAKDOWN", "NONFINITE", "ERR_INVALID_ARG", "ERR_ALLOC", "ERR_HIP",
                 "ERR_UNSUPPORTED", "BICGSTAB", "PBICGSTAB", "PBICGSTAB_RR", "CA_BICGSTAB", "CG", "CGCG",
                 "PIPE_CG", "PRECOND_NONE", "PRECOND_JACOBI", "PRECOND_JACOBI_FOLDED", "FP64", "FP32_RR64",
                 "COLS_INT32", "COLS_BLOCK16", "COLS_DIAG16", "COLS_NONE"):
        assert enum[name] == getattr(_lib, name), name
    variants = {v for k, v in enum.items() if k in ("BICGSTAB", "PBICGSTAB", "PBICGSTAB_RR", "CA_BICGSTAB", "CG",
                                                      "CGCG", "PIPE_CG")}
    assert set(solver.VARIANTS.values()) == variants
    assert set(solver.PRECISIONS.values()) == {enum["FP64"], enum["FP32_RR64"]}
    # option flags documented in the header
    assert "bit 0" in text and "bit 1" in text and "bit 2" in text
    assert (_lib.FLAG_DIRECT, _lib.FLAG_TIME_KERNELS, _lib.FLAG_ALPHA_EQ5) == (1, 2, 4)


def test_require_converged_raises_on_every_unsuccessful_status():
    """SolveFn's guard, host logic only: SUCCESS passes, MAXIT, BREAKDOWN and
    NONFINITE raise with the report attached."""
    import pytest
    from paper_1612_01395_amd import solver

    def info(status):
        return solver.SolveInfo(iters=7, n_rr=0, status=status, syncs_per_iter=2, relres_rec=1e-3,
                                relres_true=1e-3, ms=0.0, kernel_ms=(0.0, 0.0), kernel_calls=(0, 0))

    solver.require_converged(info(0), "forward")
    for st, name in ((1, "maxit"), (2, "breakdown"), (3, "nonfinite")):
        with pytest.raises(solver.NotConvergedError) as e:
            solver.require_converged(info(st), "adjoint")
        assert e.value.info.status == st and name in str(e.value) and "adjoint" in str(e.value)
