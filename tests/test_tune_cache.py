"""Host logic of the process-wide launch-shape cache (no GPU needed).

The cache maps (device, library build, rows, non-zeros, operator kind,
variant, precision, read path) to a launch shape; pbcgs_tune fills it and
solves of operators without a tuned shape of their own read it.  Here the
entries are put, replaced, refused and written to and read from JSON.
"""

import json

import pytest

from paper_1612_01395_amd import _lib, solver


def entry(**kw):
    e = {"device": "gfx950:sramecc+:xnack- 256cu", "build": "Jan  1 2026 00:00:00", "n": 2097152,
         "nnz": 14581760, "operator": "csr", "variant": "pbicgstab_rr", "precision": "fp64",
         "read_path": "default", "rows_per_wave_blocks": 8}
    e.update(kw)
    return e


@pytest.fixture(autouse=True)
def empty_cache():
    solver.tune_cache_clear()
    yield
    solver.tune_cache_clear()


def test_put_get_replace():
    assert solver.tune_cache() == []
    solver.tune_cache_put(entry())
    assert solver.tune_cache() == [entry()]
    solver.tune_cache_put(entry(rows_per_wave_blocks=16))  # same key: replaced
    assert solver.tune_cache() == [entry(rows_per_wave_blocks=16)]
    # every key field makes a new entry
    others = [entry(device="gfx942 304cu"), entry(build="other"), entry(n=2000000), entry(nnz=1),
              entry(operator="stencil7", nnz=0), entry(variant="bicgstab"), entry(precision="fp32_rr64"),
              entry(read_path="csr_arrays"), entry(read_path="int32_columns")]
    for e in others:
        solver.tune_cache_put(e)
    assert len(solver.tune_cache()) == 1 + len(others)
    assert solver.tune_cache()[1:] == others


@pytest.mark.parametrize("bad", [
    dict(rows_per_wave_blocks=3),            # not a power of two
    dict(rows_per_wave_blocks=0),
    dict(rows_per_wave_blocks=2048),         # above the largest shape
    dict(rows_per_wave_blocks=4),            # 2,048 workgroups for 2^21 rows: more than a launch takes
    dict(n=300_000_000, rows_per_wave_blocks=1),
    dict(n=0),
    dict(nnz=-1),
])
def test_put_refuses_bad_entries(bad):
    solver.tune_cache_put(entry())
    with pytest.raises(_lib.PbcgsError) as e:
        solver.tune_cache_put(entry(**bad))
    assert e.value.code == _lib.ERR_INVALID_ARG
    assert solver.tune_cache() == [entry()]


def test_put_refuses_bad_codes_and_unterminated_strings():
    lib = _lib.lib()
    base = _lib.TuneEntry()
    base.device = b"dev"
    base.build = b"b"
    base.n = 1000
    base.best = 1
    assert lib.pbcgs_tune_cache_put(_lib.ctypes.byref(base)) == 0
    for field, value in (("variant", 7), ("variant", -1), ("precision", 2), ("op_kind", 6), ("read_path", 3)):
        e = _lib.TuneEntry.from_buffer_copy(base)
        setattr(e, field, value)
        assert lib.pbcgs_tune_cache_put(_lib.ctypes.byref(e)) == _lib.ERR_INVALID_ARG, field
    e = _lib.TuneEntry.from_buffer_copy(base)
    _lib.ctypes.memmove(_lib.ctypes.addressof(e), b"x" * 64, 64)  # device without its NUL
    assert lib.pbcgs_tune_cache_put(_lib.ctypes.byref(e)) == _lib.ERR_INVALID_ARG
    assert lib.pbcgs_tune_cache_size() == 1
    out = _lib.TuneEntry()
    assert lib.pbcgs_tune_cache_get(1, _lib.ctypes.byref(out)) == _lib.ERR_INVALID_ARG
    assert lib.pbcgs_tune_cache_get(-1, _lib.ctypes.byref(out)) == _lib.ERR_INVALID_ARG
    assert lib.pbcgs_tune_cache_get(0, _lib.ctypes.byref(out)) == 0 and out.n == 1000


def test_json_round_trip(tmp_path):
    es = [entry(), entry(variant="bicgstab", rows_per_wave_blocks=16), entry(operator="convdiff27", nnz=0)]
    for e in es:
        solver.tune_cache_put(e)
    path = str(tmp_path / "sub" / "tune.json")
    assert solver.save_tune_cache(path) == 3
    doc = json.load(open(path))
    assert doc["version"] == 1 and doc["entries"] == es
    solver.tune_cache_clear()
    assert solver.load_tune_cache(path) == 3
    assert solver.tune_cache() == es


def test_load_skips_bad_entries_and_missing_files(tmp_path):
    assert solver.load_tune_cache(str(tmp_path / "none.json")) == 0
    path = tmp_path / "t.json"
    good = entry()
    doc = {"format": "pbcgs launch-shape cache", "version": 1,
           "entries": [good, entry(rows_per_wave_blocks=5), {"n": 3}, entry(variant="gmres")]}
    path.write_text(json.dumps(doc))
    assert solver.load_tune_cache(str(path)) == 1
    assert solver.tune_cache() == [good]
    path.write_text(json.dumps({"format": "something else", "entries": []}))
    with pytest.raises(ValueError):
        solver.load_tune_cache(str(path))
