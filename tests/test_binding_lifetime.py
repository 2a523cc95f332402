"""Host logic of the Python binding: a context outlives its operators.

``pbcgs_op_destroy`` uses the operator's context, so the library requires
operators to be destroyed first.  Python finalizes objects of one garbage
cycle in no fixed order; the binding therefore defers the context's
destruction until its last operator is closed.  These tests replace the
library with a recorder (no GPU needed) and check the order of the calls.
"""

import gc

import pytest

from paper_1612_01395_amd import _lib, solver


class Recorder:
    def __init__(self):
        self.calls = []

    def pbcgs_op_destroy(self, h):
        self.calls.append(("op", h))
        return 0

    def pbcgs_ctx_destroy(self, h):
        self.calls.append(("ctx", h))
        return 0


@pytest.fixture
def rec(monkeypatch):
    r = Recorder()
    monkeypatch.setattr(_lib, "lib", lambda: r)
    return r


def fake_context(handle):
    ctx = object.__new__(solver.Context)
    ctx._live_ops = 0
    ctx._closing = False
    ctx.handle = handle
    return ctx


def test_context_close_waits_for_its_operators(rec):
    ctx = fake_context("C")
    a = solver.Operator(ctx, "A", 4, (), "csr")
    b = solver.Operator(ctx, "B", 4, (), "csr")
    ctx.close()
    assert rec.calls == []
    a.close()
    assert rec.calls == [("op", "A")]
    b.close()
    assert rec.calls == [("op", "A"), ("op", "B"), ("ctx", "C")]
    ctx.close()  # idempotent
    b.close()
    assert len(rec.calls) == 3


def test_context_without_operators_closes_at_once(rec):
    ctx = fake_context("C")
    ctx.close()
    assert rec.calls == [("ctx", "C")]


def test_garbage_cycle_destroys_operators_first(rec):
    for _ in range(20):  # the collector's order within a cycle is not fixed: try several
        rec.calls.clear()
        ctx = fake_context("C")
        op = solver.Operator(ctx, "O", 4, (), "csr")
        holder = {"op": op, "ctx": ctx}
        holder["self"] = holder  # a reference cycle holding both
        ctx.cycle = holder
        del ctx, op, holder
        gc.collect()
        assert rec.calls == [("op", "O"), ("ctx", "C")]
