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


# ---------------------------------------------------------------------------
# The precision form, every operation rounded as an IEEE machine rounds it.
# ---------------------------------------------------------------------------

def _pairwise(vals, rnd):
    """Balanced-tree sum of a power-of-two number of values, each addition
    rounded by ``rnd``."""
    if len(vals) == 1:
        return vals[0]
    h = len(vals) // 2
    return rnd(_pairwise(vals[:h], rnd) + _pairwise(vals[h:], rnd))


def _dot_rounded(u, v, rnd):
    """Rounded products, zero-padded to a power of two, summed pairwise with
    every addition rounded; the final + 0 only normalises a signed zero."""
    prods = [rnd(a * b) for a, b in zip(u, v)]
    size = 1
    while size < len(prods):
        size *= 2
    prods += [ZERO] * (size - len(prods))
    return _pairwise(prods, rnd)


def _spmv_rounded(A, x, rnd):
    """Each row summed in stored order from 0, product and sum rounded."""
    out = []
    for row in A:
        acc = ZERO
        for c, a in row:
            acc = rnd(acc + rnd(a * x[c]))
        out.append(acc)
    return out


def pbicgstab_mp(A, b, x0, *, tol, maxit, rr_period=0, rr_max=-1, reading=()):
    """Precision form of p-BiCGStab with residual replacement, with every
    operation an exactly computed rational rounded once to binary32 or
    binary64 (:mod:`oracle.ieee`).

    ``A`` holds binary64 values (rows of ``(col, Fraction)``), ``b`` and
    ``x0`` binary64 vectors.  The reading of the precision form followed here:
    binary32 operator f(A), vectors, recurrences and dot products (pairwise,
    binary32 additions, widened afterwards); alpha, beta, omega in binary64
    from the widened dots, passed to the vector updates rounded to binary32;
    x updated in binary64 from the binary32 p and q; every replacement step in
    binary64 on A and x, rounded once when stored: r = f(b - A x),
    w = f(A (b - A x)) in the iteration that replaces, s = f(A p),
    z = f(A (A p)) at the start of the next one (Section 4.2 placement "C");
    the setup is such a replacement and rho_0 = sqrt((r_0, r_0)) with the
    binary32 dot.  A binary32 recursive residual at or below tol is confirmed
    by the binary64 ||b - A x|| / rho_0; if that is above tol the iteration
    replaces r and w, reduces again and goes on without a second stop test.

    ``reading`` names deliberate departures, used to show that the tests can
    tell them apart: ``"scalars64"`` (the vector updates use the unrounded
    binary64 scalars, in binary64, rounded when stored), ``"w_of_rounded_r"``
    (a replacement forms w from the rounded binary32 r instead of the binary64
    one), ``"rho0_64"`` (rho_0 from the binary64 residual).

    Returns ``(x, info)`` with ``info`` = iters, n_rr, status ("success",
    "maxit", "breakdown"), relres_rec, relres_true and the history of the
    recursive relative residuals.
    """
    from oracle.ieee import round32 as f32, round64 as f64, sqrt64

    alt = set(reading)
    unknown = alt - {"scalars64", "w_of_rounded_r", "rho0_64"}
    if unknown:
        raise ValueError(f"unknown readings {sorted(unknown)}")
    n = len(b)
    A32 = [[(c, f32(a)) for c, a in row] for row in A]
    tol = Fraction(tol)
    x = [Fraction(v) for v in x0]
    b = [Fraction(v) for v in b]

    def spmv64(v):
        return _spmv_rounded(A, v, f64)

    def spmv32(v):
        return _spmv_rounded(A32, v, f32)

    def dot32(u, v):
        return _dot_rounded(u, v, f32)

    def true_residual64():
        ax = spmv64(x)
        return [f64(bi - ai) for bi, ai in zip(b, ax)]

    def replace_r_w():
        """r = f(b - A x), w = f(A (b - A x)): binary64 steps, rounded when stored."""
        res64 = true_residual64()
        r_new = [f32(v) for v in res64]
        w64 = spmv64(r_new if "w_of_rounded_r" in alt else res64)
        return r_new, [f32(v) for v in w64], res64

    def upd(base, sc, other, sc2=None, third=None):
        """base + sc (other - sc2 third), or base - sc other when sc2 is None,
        with the scalars as the vector updates see them."""
        if "scalars64" in alt:
            rnd = f64
        else:
            rnd = f32
        if sc2 is None:
            return [f32(rnd(bv - rnd(sc * ov))) for bv, ov in zip(base, other)]
        return [f32(rnd(bv + rnd(sc * rnd(ov - rnd(sc2 * tv))))) for bv, ov, tv in zip(base, other, third)]

    def scal(v):
        return v if "scalars64" in alt else f32(v)

    info = {"iters": 0, "n_rr": 0, "status": "maxit", "relres_rec": Fraction(1), "history": [Fraction(1)]}

    def finish(status):
        info["status"] = status
        res = true_residual64()
        nr = _dot_rounded(res, res, f64)
        info["relres_true"] = f64(sqrt64(nr) / rho0) if rho0 > 0 else ZERO
        return x, info

    # setup (a replacement): r_0, w_0, t_0 = A w_0, rho_0, alpha_0
    r, w, res64 = replace_r_w()
    r0 = list(r)
    gamma = dot32(r0, r0)
    rho0 = sqrt64(_dot_rounded(res64, res64, f64)) if "rho0_64" in alt else sqrt64(gamma)
    if rho0 == 0:
        info["relres_rec"] = ZERO
        return finish("success")
    t = spmv32(w)
    delta = dot32(r0, w)
    if delta == 0:
        return finish("breakdown")
    alpha, beta, omega = f64(gamma / delta), ZERO, ZERO
    p = [ZERO] * n
    s = [ZERO] * n
    z = [ZERO] * n
    v = [ZERO] * n
    pending = False
    n_rr = 0

    for i in range(maxit):
        af, bf, wf = scal(alpha), scal(beta), scal(omega)
        # search direction, then s and z: by recurrence, or (after a
        # replacement) recomputed in binary64 from the new p
        p = upd(r, bf, p, wf, s)
        if pending:
            s64 = spmv64(p)
            s = [f32(e) for e in s64]
            z = [f32(e) for e in spmv64(s64)]
            pending = False
        else:
            s, z = upd(w, bf, s, wf, z), upd(t, bf, z, wf, v)
        # q, y; reduction 1; v = A z
        q = upd(r, af, s)
        y = upd(w, af, z)
        th1, th2 = dot32(q, y), dot32(y, y)
        v = spmv32(z)
        if th2 == 0:
            x = [f64(xi + f64(alpha * pi)) for xi, pi in zip(x, p)]
            info["iters"] = i + 1
            info["relres_rec"] = ZERO
            info["history"].append(ZERO)
            return finish("success")
        omega = f64(th1 / th2)
        wn = scal(omega)
        # binary64 x; binary32 r and w recurrences
        x = [f64(f64(xi + f64(alpha * pi)) + f64(omega * qi)) for xi, pi, qi in zip(x, p, q)]
        r = upd(q, wn, y)
        tav = upd(t, af, v)
        w = upd(y, wn, tav)
        info["iters"] = i + 1
        forced = False
        replace = rr_period > 0 and (i + 1) % rr_period == 0 and (rr_max < 0 or (i + 1) // rr_period <= rr_max)
        while True:
            if replace:
                r, w, _ = replace_r_w()
                pending = True
                n_rr += 1
                info["n_rr"] = n_rr
                replace = False
            # reduction 2 and the stopping test
            g1, eta, sig_s, sig_z, nu = dot32(r0, r), dot32(r0, w), dot32(r0, s), dot32(r0, z), dot32(r, r)
            rel = f64(sqrt64(nu) / rho0)
            info["relres_rec"] = rel
            if len(info["history"]) == i + 2:
                info["history"][i + 1] = rel
            else:
                info["history"].append(rel)
            if rel <= tol and not forced:
                res = true_residual64()
                if f64(sqrt64(_dot_rounded(res, res, f64)) / rho0) <= tol:
                    return finish("success")
                forced = True
                replace = True
                continue
            break
        t = spmv32(w)
        if omega == 0 or gamma == 0:
            return finish("breakdown")
        beta = f64(f64(alpha / omega) * f64(g1 / gamma))
        den = f64(f64(eta + f64(beta * sig_s)) - f64(f64(beta * omega) * sig_z))
        if den == 0 or g1 == 0:
            return finish("breakdown")
        alpha = f64(g1 / den)
        gamma = g1
    return finish("maxit")
