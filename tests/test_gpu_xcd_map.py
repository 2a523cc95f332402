"""GPU parity of the XCD-contiguous workgroup indices (``PBCGS_XCD_MAP``).

The map deals the indices of a launch so that each of the 8 XCDs runs one
contiguous run of them; every index keeps its rows and its partial-sum slot,
so every solve must equal the oracle bit for bit with the map on and off,
for every variant, at workgroup counts that are and are not multiples of 8
(runs of unequal length), and at one workgroup.
"""

import numpy as np
import pytest

import oracle
from paper_1612_01395_amd import inputs, solver
from gpu_util import csr_op, dev_t, host, require_gpu, same, say

pytestmark = pytest.mark.gpu

ALG = {"bicgstab": oracle.ALG_BICGSTAB, "pbicgstab": oracle.ALG_PBICGSTAB, "pbicgstab_rr": oracle.ALG_PBICGSTAB_RR,
       "ca_bicgstab": oracle.ALG_CA_BICGSTAB, "cg": oracle.ALG_CG, "cgcg": oracle.ALG_CGCG,
       "pipe_cg": oracle.ALG_PIPE_CG}


@pytest.mark.parametrize("gtarget", [1, 3, 10, 64, 1023])
@pytest.mark.parametrize("variant", list(ALG))
def test_xcd_map_bitwise(variant, gtarget, monkeypatch):
    require_gpu()
    monkeypatch.setenv("PBCGS_GTARGET", str(gtarget))
    cg = variant in ("cg", "cgcg", "pipe_cg")
    A = oracle.assemble_workload(inputs.workload("c2s" if cg else "c2", n=40))
    precond = "jacobi" if cg else "jacobi_folded"
    b = oracle.spmv(A, inputs.x_true(A.n))
    d = oracle.jacobi_dinv(A)
    kw = dict(tol=1e-10, maxit=800, rr_period=17)
    if precond == "jacobi_folded":
        x_or, i_or = oracle.solve_folded(A, b, algo=ALG[variant], dinv=d, history=True, **kw)
    else:
        x_or, i_or = oracle.solve(A, b, algo=ALG[variant], dinv=d, history=True, **kw)
    op = csr_op(A)
    for xmap in ("1", "0"):
        monkeypatch.setenv("PBCGS_XCD_MAP", xmap)
        say(f"xcd map {xmap}: {variant} gtarget={gtarget}")
        x, info = solver.solve(op, dev_t(b), variant=variant, precond=precond, history=True, **kw)
        assert (info.status, info.iters, info.n_rr) == (i_or["status"], i_or["iters"], i_or["n_rr"]), (info, i_or)
        assert same(host(x), x_or), float(np.abs(host(x) - x_or).max())
        assert same(host(info.history), i_or["history"])
