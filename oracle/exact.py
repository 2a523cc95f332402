"""Exact rational twins of the paper's BiCGStab variants -- TEST INFRASTRUCTURE ONLY.

Every quantity is a ``fractions.Fraction``; nothing is rounded.  The tests use
these to pin the FP64 oracle against facts the paper states for exact
arithmetic (arXiv 1612.01395):

* Algorithm 7 (BiCGStab), Algorithm 8 (CA-BiCGStab) and Algorithm 9
  (p-BiCGStab) produce the same iterates (Sections 3.2-3.3);
* Algorithm 10 (preconditioned BiCGStab) and Algorithm 11 (preconditioned
  p-BiCGStab) produce the same iterates (Section 3.6);
* residual replacement (Section 4.2) replaces vectors by values equal to
  them, so it changes nothing;
* like BiCG, BiCGStab reaches the exact solution in at most N steps unless a
  denominator vanishes first.

Matrices are lists of rows, each row a list of ``(col, Fraction)`` pairs.
Each function returns a list of per-iteration records
``{"x": x_{i+1}, "r": r_{i+1}, "alpha": a_i, "omega": w_i, "beta": b_i}``
and a final status string.
"""

from __future__ import annotations

from fractions import Fraction

ZERO = Fraction(0)


def matvec(A, x):
    return [sum((v * x[c] for c, v in row), ZERO) for row in A]


def dot(a, b):
    return sum((p * q for p, q in zip(a, b)), ZERO)


def axpy(a, x, y):
    """y + a x."""
    return [yi + a * xi for xi, yi in zip(x, y)]


def sub(x, y):
    return [a - b for a, b in zip(x, y)]


def scale(d, x):
    return [a * b for a, b in zip(d, x)]


def _rec(x, r, alpha, omega, beta):
    return {"x": list(x), "r": list(r), "alpha": alpha, "omega": omega, "beta": beta}


def bicgstab(A, b, x0, maxit, dinv=None):
    """Algorithm 7; with ``dinv`` (M^{-1} = diag(dinv)) Algorithm 10."""
    n = len(b)
    M = (lambda v: scale(dinv, v)) if dinv is not None else (lambda v: list(v))
    x = list(x0)
    r0 = sub(b, matvec(A, x))
    r = list(r0)
    p = list(r0)
    out = []
    for _ in range(maxit):
        if all(v == 0 for v in r):
            return out, "converged"
        ph = M(p)
        s = matvec(A, ph)
        rs = dot(r0, s)
        if rs == 0:
            return out, "breakdown"
        alpha = dot(r0, r) / rs
        q = axpy(-alpha, s, r)
        qh = M(q)
        y = matvec(A, qh)
        yy = dot(y, y)
        if yy == 0:
            x = [xi + alpha * pi for xi, pi in zip(x, ph)]
            out.append(_rec(x, [ZERO] * n, alpha, None, None))
            return out, "converged"
        omega = dot(q, y) / yy
        x = [xi + alpha * pi + omega * qi for xi, pi, qi in zip(x, ph, qh)]
        r_new = axpy(-omega, y, q)
        if omega == 0:
            out.append(_rec(x, r_new, alpha, omega, None))
            return out, "breakdown"
        beta = (alpha / omega) * (dot(r0, r_new) / dot(r0, r))
        p = [ri + beta * (pi - omega * si) for ri, pi, si in zip(r_new, p, s)]
        r = r_new
        out.append(_rec(x, r, alpha, omega, beta))
    return out, "maxit"


def ca_bicgstab(A, b, x0, maxit, alpha_form=3):
    """Algorithm 8 (communication-avoiding BiCGStab), unpreconditioned;
    ``alpha_form`` 5 takes alpha_{i+1} from eq. (5)."""
    n = len(b)
    x = list(x0)
    r0 = sub(b, matvec(A, x))
    r = list(r0)
    w = matvec(A, r)
    rw = dot(r0, w)
    if all(v == 0 for v in r):
        return [], "converged"
    if rw == 0:
        return [], "breakdown"
    alpha = dot(r0, r0) / rw
    beta = ZERO
    omega = ZERO
    p = [ZERO] * n
    s = [ZERO] * n
    z = [ZERO] * n
    out = []
    for _ in range(maxit):
        p = [ri + beta * (pi - omega * si) for ri, pi, si in zip(r, p, s)]
        s = [wi + beta * (si - omega * zi) for wi, si, zi in zip(w, s, z)]
        z = matvec(A, s)
        q = axpy(-alpha, s, r)
        y = axpy(-alpha, z, w)
        yy = dot(y, y)
        if yy == 0:
            x = [xi + alpha * pi for xi, pi in zip(x, p)]
            out.append(_rec(x, [ZERO] * n, alpha, None, None))
            return out, "converged"
        omega = dot(q, y) / yy
        x = [xi + alpha * pi + omega * qi for xi, pi, qi in zip(x, p, q)]
        r_new = axpy(-omega, y, q)
        w = matvec(A, r_new)
        g1, g0 = dot(r0, r_new), dot(r0, r)
        if all(v == 0 for v in r_new):
            out.append(_rec(x, r_new, alpha, omega, None))
            return out, "converged"
        beta = (alpha / omega) * (g1 / g0)
        if alpha_form == 5:
            if g1 == 0:
                out.append(_rec(x, r_new, alpha, omega, beta))
                return out, "breakdown"
            den = (1 / omega + dot(r0, w) / g1) - (beta * omega) * (dot(r0, z) / g1)
            num = 1
        else:
            den = dot(r0, w) + beta * dot(r0, s) - beta * omega * dot(r0, z)
            num = g1
        out.append(_rec(x, r_new, alpha, omega, beta))
        r = r_new
        if den == 0:
            return out, "breakdown"
        alpha = num / den
    return out, "maxit"


def pbicgstab(A, b, x0, maxit, dinv=None, rr_period=0, alpha_form=3):
    """Algorithm 9; with ``dinv`` Algorithm 11.  ``rr_period`` > 0 adds the
    residual replacement of Section 4.2 (same placement as the FP64 oracle).
    ``alpha_form`` 5 takes alpha_{i+1} from eq. (5) instead of eq. (3)."""
    n = len(b)
    pc = dinv is not None
    M = (lambda v: scale(dinv, v)) if pc else (lambda v: list(v))
    x = list(x0)
    r0 = sub(b, matvec(A, x))
    r = list(r0)
    if all(v == 0 for v in r):
        return [], "converged", []
    rh = M(r)
    w = matvec(A, rh)
    wh = M(w)
    t = matvec(A, wh)
    rw = dot(r0, w)
    if rw == 0:
        return [], "breakdown", []
    gamma = dot(r0, r0)
    alpha = gamma / rw
    beta = ZERO
    omega = ZERO
    ph = [ZERO] * n
    s = [ZERO] * n
    sh = [ZERO] * n
    z = [ZERO] * n
    zh = [ZERO] * n
    v = [ZERO] * n
    out = []
    replaced = []  # (iteration, max |true - recursive| over the replaced vectors)
    rr_pending = False
    for i in range(maxit):
        ph = [a + beta * (c - omega * d) for a, c, d in zip(rh, ph, sh)]
        if rr_pending:
            s_true = matvec(A, ph)
            sh_true = M(s_true)
            z_true = matvec(A, sh_true)
            s_rec = [a + beta * (c - omega * d) for a, c, d in zip(w, s, z)]
            sh_rec = [a + beta * (c - omega * d) for a, c, d in zip(wh, sh, zh)] if pc else s_rec
            z_rec = [a + beta * (c - omega * d) for a, c, d in zip(t, z, v)]
            gap = max(abs(a - c) for a, c in zip(s_true + sh_true + z_true, s_rec + sh_rec + z_rec))
            replaced.append((i, "s,s^,z", gap))
            s, sh, z = s_true, sh_true, z_true
            rr_pending = False
        else:
            s_new = [a + beta * (c - omega * d) for a, c, d in zip(w, s, z)]
            sh_new = [a + beta * (c - omega * d) for a, c, d in zip(wh, sh, zh)] if pc else s_new
            z = [a + beta * (c - omega * d) for a, c, d in zip(t, z, v)]
            s, sh = s_new, sh_new
        q = axpy(-alpha, s, r)
        qh = axpy(-alpha, sh, rh) if pc else q
        y = axpy(-alpha, z, w)
        yy = dot(y, y)
        qy = dot(q, y)
        zh = M(z)
        v = matvec(A, zh)
        if yy == 0:
            x = [xi + alpha * pi for xi, pi in zip(x, ph)]
            out.append(_rec(x, [ZERO] * n, alpha, None, None))
            return out, "converged", replaced
        omega = qy / yy
        x = [xi + alpha * pi + omega * qi for xi, pi, qi in zip(x, ph, qh)]
        r = axpy(-omega, y, q)
        rh = [a - omega * (c - alpha * d) for a, c, d in zip(qh, wh, zh)] if pc else r
        w = [a - omega * (c - alpha * d) for a, c, d in zip(y, t, v)]
        if rr_period > 0 and (i + 1) % rr_period == 0:
            r_true = sub(b, matvec(A, x))
            rh_true = M(r_true)
            w_true = matvec(A, rh_true)
            gap = max(abs(a - c) for a, c in zip(r_true + rh_true + w_true, r + rh + w))
            replaced.append((i, "r,r^,w", gap))
            r, rh, w = r_true, rh_true, w_true
            rr_pending = True
        g1 = dot(r0, r)
        eta = dot(r0, w)
        ss = dot(r0, s)
        sz = dot(r0, z)
        if all(c == 0 for c in r):
            out.append(_rec(x, r, alpha, omega, None))
            return out, "converged", replaced
        wh = M(w)
        t = matvec(A, wh)
        if omega == 0:
            out.append(_rec(x, r, alpha, omega, None))
            return out, "breakdown", replaced
        beta = (alpha / omega) * (g1 / gamma)
        out.append(_rec(x, r, alpha, omega, beta))
        if alpha_form == 5:
            if g1 == 0:
                return out, "breakdown", replaced
            den = (1 / omega + eta / g1) - (beta * omega) * (sz / g1)
            if den == 0:
                return out, "breakdown", replaced
            alpha = 1 / den
        else:
            den = eta + beta * ss - beta * omega * sz
            if den == 0:
                return out, "breakdown", replaced
            alpha = g1 / den
        gamma = g1
    return out, "maxit", replaced


# ---------------------------------------------------------------------------
# The CG family of Section 2 (symmetric positive definite A).  Each record
# holds x_{i+1}, r_{i+1}, alpha_i and the beta_i that built p_i (0 for i = 0),
# so the three algorithms can be compared record by record.
# ---------------------------------------------------------------------------

def cg(A, b, x0, maxit, dinv=None):
    """Algorithm 2 (standard preconditioned CG)."""
    M = (lambda v: scale(dinv, v)) if dinv is not None else (lambda v: list(v))
    x = list(x0)
    r = sub(b, matvec(A, x))
    if all(v == 0 for v in r):
        return [], "converged"
    u = M(r)
    p = list(u)
    gamma = dot(r, u)
    beta = ZERO
    out = []
    for _ in range(maxit):
        s = matvec(A, p)
        delta = dot(s, p)
        if delta == 0:
            return out, "breakdown"
        alpha = gamma / delta
        x = axpy(alpha, p, x)
        r = axpy(-alpha, s, r)
        u = M(r)
        out.append(_rec(x, r, alpha, None, beta))
        if all(v == 0 for v in r):
            return out, "converged"
        gamma1 = dot(r, u)
        beta = gamma1 / gamma
        p = axpy(beta, p, u)
        gamma = gamma1
    return out, "maxit"


def cgcg(A, b, x0, maxit, dinv=None):
    """Algorithm 4 (Chronopoulos & Gear CG)."""
    n = len(b)
    M = (lambda v: scale(dinv, v)) if dinv is not None else (lambda v: list(v))
    x = list(x0)
    r = sub(b, matvec(A, x))
    if all(v == 0 for v in r):
        return [], "converged"
    u = M(r)
    w = matvec(A, u)
    gamma, delta = dot(r, u), dot(w, u)
    if delta == 0:
        return [], "breakdown"
    alpha, beta = gamma / delta, ZERO
    p = [ZERO] * n
    s = [ZERO] * n
    out = []
    for _ in range(maxit):
        p = axpy(beta, p, u)
        s = axpy(beta, s, w)
        x = axpy(alpha, p, x)
        r = axpy(-alpha, s, r)
        u = M(r)
        w = matvec(A, u)
        out.append(_rec(x, r, alpha, None, beta))
        if all(v == 0 for v in r):
            return out, "converged"
        gamma1, delta = dot(r, u), dot(w, u)
        if gamma1 == 0:
            return out, "breakdown"
        beta = gamma1 / gamma
        den = delta / gamma1 - beta / alpha
        if den == 0:
            return out, "breakdown"
        alpha = 1 / den
        gamma = gamma1
    return out, "maxit"


def pipe_cg(A, b, x0, maxit, dinv=None):
    """Algorithm 6 (pipelined CG)."""
    n = len(b)
    M = (lambda v: scale(dinv, v)) if dinv is not None else (lambda v: list(v))
    x = list(x0)
    r = sub(b, matvec(A, x))
    if all(v == 0 for v in r):
        return [], "converged"
    u = M(r)
    w = matvec(A, u)
    z = [ZERO] * n
    q = [ZERO] * n
    s = [ZERO] * n
    p = [ZERO] * n
    alpha = gamma = None
    out = []
    for i in range(maxit):
        gamma1, delta = dot(r, u), dot(w, u)
        m = M(w)
        nv = matvec(A, m)
        if i == 0:
            if delta == 0:
                return out, "breakdown"
            beta, alpha = ZERO, gamma1 / delta
        else:
            if gamma1 == 0:
                return out, "breakdown"
            beta = gamma1 / gamma
            den = delta / gamma1 - beta / alpha
            if den == 0:
                return out, "breakdown"
            alpha = 1 / den
        gamma = gamma1
        z = axpy(beta, z, nv)
        q = axpy(beta, q, m)
        s = axpy(beta, s, w)
        p = axpy(beta, p, u)
        x = axpy(alpha, p, x)
        r = axpy(-alpha, s, r)
        u = axpy(-alpha, q, u)
        w = axpy(-alpha, z, w)
        out.append(_rec(x, r, alpha, None, beta))
        if all(v == 0 for v in r):
            return out, "converged"
    return out, "maxit"
