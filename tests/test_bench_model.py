"""CPU checks of the benchmark's bookkeeping: the algorithmic byte model the
roofline divides by, and the source hash that decides whether the recorded
HBM traffic still describes the kernels."""

import json

import bench

N, NNZ = 2097152, 14581760          # 3-D 7-point 128^3
VEC, MAT = 8 * N, 4 * (N + 1) + 12 * NNZ


def test_fused_kernel_bytes_at_128():
    ka, kb, it = bench.algorithmic_bytes(N, NNZ, "pbicgstab", False)
    assert (ka, kb) == (MAT + 10 * VEC, MAT + 12 * VEC) == (351141892, 384696324)
    assert it == 2 * MAT + 22 * VEC
    # BiCGStab 19 passes folded, 23 with the hatted vectors; literal Algorithm 11 34
    assert bench.algorithmic_bytes(N, NNZ, "bicgstab", False)[2] == 2 * MAT + 19 * VEC
    assert bench.algorithmic_bytes(N, NNZ, "bicgstab", False, folded=False)[2] == 2 * MAT + 23 * VEC
    assert bench.algorithmic_bytes(N, NNZ, "pbicgstab", False, folded=False)[2] == 2 * MAT + 34 * VEC
    assert bench.algorithmic_bytes(N, NNZ, "ca_bicgstab", False)[2] == 2 * MAT + 24 * VEC
    assert bench.algorithmic_bytes(N, NNZ, "pbicgstab", True)[2] == 22 * VEC  # stencil: no operator bytes


def test_compact_column_bytes_at_128():
    """With the int16 column copy each non-zero costs 10 bytes instead of 12."""
    mat16 = 4 * (N + 1) + 10 * NNZ
    ka, kb, it = bench.algorithmic_bytes(N, NNZ, "pbicgstab", False, index_bytes=2)
    assert (ka, kb) == (mat16 + 10 * VEC, mat16 + 12 * VEC) == (321978372, 355532804)
    assert it == 2 * mat16 + 22 * VEC
    assert bench.algorithmic_bytes(N, NNZ, "pbicgstab", True, index_bytes=2)[2] == 22 * VEC
    assert bench.algorithmic_bytes_cg(N, NNZ, "pipe_cg", True, 2) == mat16 + 18 * VEC


def test_cg_family_bytes():
    for variant, passes in (("cg", 12), ("cgcg", 14), ("pipe_cg", 18)):
        assert bench.algorithmic_bytes_cg(N, NNZ, variant, True) == MAT + passes * VEC


def test_code_text_ignores_comments_only():
    src = 'int a = 1; // note\n/* block\n comment */ int b = 2;\nconst char* s = "x // y /* z */";\nchar c = \'/\';\n'
    code = bench.code_text(src)
    assert "note" not in code and "block" not in code
    assert '"x // y /* z */"' in code and "'/'" in code
    assert bench.code_text(src.replace("// note", "// other note")) == code
    assert bench.code_text(src.replace("int b = 2", "int b = 3")) != code


def test_recorded_traffic_matches_the_sources():
    """The committed counter summary was taken on the current kernels (after a
    kernel change the benchmark reports no traffic until the counters are
    taken again; this test then skips with that reason).  Every recorded
    launch grid moved at least the algorithmic bytes and at most 25 % more
    (the excess is re-reads of the gathered vector's neighbours a plane
    away, 15-40 MB per launch at 128^3; with the value-coded operator the
    algorithmic bytes are smallest, so the same excess is up to 20 % of
    them)."""
    import pytest
    with open(bench.TRAFFIC_FILE) as f:
        t = json.load(f)
    if t["source_hash"] != bench.kernel_source_hash():
        pytest.skip("kernel sources changed since the HBM counters were taken")
    nd = t["diagonals"]
    for k in ("k_pa", "k_pb"):
        algo = bench.algorithmic_bytes(N, NNZ, "pbicgstab", False, dia=nd,
                                       codes=t.get("value_codes", False))[0 if k == "k_pa" else 1]
        grids = t["bytes_per_launch"][k]
        assert grids
        for g in grids:
            got = bench.measured_traffic(k, int(g))
            assert got is not None and algo < got < 1.25 * algo, (k, g, got, algo)
        assert bench.measured_traffic(k, 12345) is None


def test_diagonal_layout_bytes_at_128():
    """Read through its diagonal layout the 7-point operator costs a 4-byte
    mask and 7 values (8 bytes each) per row: 60 bytes per row and product,
    against 4 + 10 nnz/N = 73.5 with the compact CSR stream."""
    ka, kb, it = bench.algorithmic_bytes(N, NNZ, "pbicgstab", False, dia=7)
    assert (ka, kb) == (60 * N + 10 * VEC, 60 * N + 12 * VEC) == (293601280, 327155712)
    assert it == 2 * 60 * N + 22 * VEC
    assert bench.algorithmic_bytes_cg(N, NNZ, "pipe_cg", True, dia=7) == 60 * N + 18 * VEC


def test_value_coded_layout_bytes_at_128():
    """With value indexing the operator is one 8-byte word of codes per row
    and a 16-entry binary64 table per diagonal, whatever the row's entries."""
    ka, kb, it = bench.algorithmic_bytes(N, NNZ, "pbicgstab", False, dia=7, codes=True)
    tabs = 7 * 16 * 8
    assert (ka, kb) == (8 * N + tabs + 10 * VEC, 8 * N + tabs + 12 * VEC) == (184550272, 218104704)
    assert it == 2 * (8 * N + tabs) + 22 * VEC
    b1, b3, itb = bench.algorithmic_bytes(N, NNZ, "bicgstab", False, dia=7, codes=True)
    assert (b1, b3, itb) == (8 * N + tabs + 3 * VEC, 8 * N + tabs + 2 * VEC, 2 * (8 * N + tabs) + 19 * VEC)
    assert bench.algorithmic_bytes_cg(N, NNZ, "pipe_cg", True, dia=7, codes=True) == 8 * N + tabs + 18 * VEC
    # codes only change the bytes of a diagonal layout
    assert bench.algorithmic_bytes(N, NNZ, "pbicgstab", False, codes=True) == \
        bench.algorithmic_bytes(N, NNZ, "pbicgstab", False)


def test_matrix_free_27_point_bytes_at_256():
    """The matrix-free 27-point product reads the (n+1)^3 cell coefficients and
    gathers dinv (folded Jacobi) besides its input vector."""
    n = 256
    Nn = n ** 3
    mat = 8 * (n + 1) ** 3 + 8 * Nn
    ka, kb, it = bench.algorithmic_bytes_mf27(n, "pbicgstab_rr")
    assert (ka, kb) == (mat + 10 * 8 * Nn, mat + 12 * 8 * Nn)
    assert it == 2 * mat + 22 * 8 * Nn
    assert bench.algorithmic_bytes_mf27(n, "bicgstab")[2] == 2 * mat + 19 * 8 * Nn
