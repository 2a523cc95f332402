"""Benchmark: p-BiCGStab(+RR) iterations/s and HBM bandwidth on one MI355X,
against plain BiCGStab on the same GPU.

Workload (the metric's configuration): 3-D 7-point first-order upwind
convection-diffusion on a 128^3 grid (2,097,152 unknowns, 14,581,760
non-zeros), h^2-scaled, beta = (50, 30, 10), CSR FP64, Jacobi, x_true ~ U[0,1)
(seed 1), b = A x_true, x0 = 0, tol 1e-8 on ||r_i||/||r_0||, residual
replacement every 50 iterations.  Inputs are synthetic and resident in HBM
before the timed region.

Jacobi is right preconditioning (A M^{-1} y = b, x = M^{-1} y).  The headline
runs it with A M^{-1} formed once per solve, so the unpreconditioned
p-BiCGStab (Algorithm 9) iterates on it; the literal Algorithm 11 (M^{-1}
applied to hatted vectors) and the two forms of plain BiCGStab (Algorithm 7 on
A M^{-1}, Algorithm 10) are timed beside it on the same kernels.

One step = one complete solve (forming A M^{-1}, setup, every iteration, the
replacements, x = M^{-1} y and the final true-residual check).  value =
iterations / second over the timed steps.  Prints one JSON line.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_pb_c2.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1612_01395_amd", "csrc", "kernels.hpp")]  # every solver kernel


def code_text(src: str) -> str:
    """The source with comments and blank lines removed (string literals kept),
    so that editing a comment does not count as changing a kernel."""
    out, i, n = [], 0, len(src)
    while i < n:
        c = src[i]
        if src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            i = n if j < 0 else j + 2
        elif c in "\"'":
            j = i + 1
            while j < n and src[j] != c:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        else:
            out.append(c)
            i += 1
    return "\n".join(line.rstrip() for line in "".join(out).splitlines() if line.strip())


def kernel_source_hash() -> str:
    """Hash of the code (without comments) of the kernel source."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, encoding="utf-8") as fh:
            h.update(code_text(fh.read()).encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, grid_threads: int):
    """HBM bytes per launch of `kernel` at a grid of `grid_threads` threads
    from the committed rocprofv3 counter summary (FETCH_SIZE and WRITE_SIZE,
    each scaled by the same counter's reading for a plain copy of known
    size), or None if the kernel source changed since the counters were taken
    or the grid was not measured."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != kernel_source_hash():
        return None
    return t.get("bytes_per_launch", {}).get(kernel, {}).get(str(grid_threads))


def progress(msg: str) -> None:
    """One line on stderr when a leg of the benchmark ends."""
    sys.stderr.write(f"[bench] {msg}\n")
    sys.stderr.flush()


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--n", type=int, default=128, help="grid side of the 3-D workload")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=12.0, help="target length of the oracle sample")
    p.add_argument("--only", default="",
                   help="comma list of legs to run: pipe,index32,bicg,explicit,stencil,fixed,cg,precision,batched,sweep,paper,"
                        "configs")
    p.add_argument("--configs", default="c1,c3", help="comma list of the configs the configs leg runs")
    p.add_argument("--copy-calib", action="store_true",
                   help="also run a plain 256 MiB device copy (to calibrate HBM byte counters)")
    p.add_argument("--tune-cache", default=os.environ.get("PBCGS_TUNE_CACHE",
                                                           os.path.join(os.path.expanduser("~"), ".cache", "pbcgs",
                                                                        "tune.json")),
                   help="JSON file of tuned launch shapes: read before tuning, written after ('' = none)")
    p.add_argument("--retune", action="store_true", help="tune every leg even where the cache holds its shape")
    p.add_argument("--cpu-child", action="store_true", help=argparse.SUPPRESS)  # the oracle timing process
    return p.parse_args()


def algorithmic_bytes(N: int, nnz: int, variant: str, stencil: bool, folded: bool = True, index_bytes: int = 4,
                      dia: int = 0, codes: bool = False):
    """Algorithmic HBM bytes of the two dominant kernels of one iteration and
    of the whole iteration: (K_a, K_b, iteration).

    Every array a kernel touches is counted once: the operator (int32
    row_ptr, the column indices at `index_bytes` each -- 2 for the compact
    int16 copy, 4 for int32 columns -- and f64 val; nothing for the stencil)
    and one read or write of each N-vector (the gathered SpMV input counted
    once).  Jacobi
    with a constant diagonal is a scalar (no dinv vector).  With ``dia`` > 0
    the operator is read through its diagonal layout instead: a 4-byte mask per
    row and one 8-byte value per diagonal and row (absent entries' slots
    included); with ``codes`` (value indexing, ``SolveInfo.value_codes``) an
    8-byte word of one-byte codes per row and each diagonal's 16-entry table.

    Folded Jacobi (A M^{-1} formed, Algorithm 9 on it): K_a reads w, r, v, s,
    z, p and writes p, s, t, z (10 vectors); K_b reads z, r, s, w, t, x, p, r0
    and writes x, v, r, w (12): 22 per iteration.  Literal Algorithm 11: K_a
    reads w^, r, w, v, s, z, r^, s^, z^, p^ and writes p^, s^, s, t, z, z^ (16);
    K_b reads z^, r, s, w, z, t, r^, s^, w^, x, p^, r0 and writes x, v, r, r^,
    w, w^ (18): 34.  BiCGStab, SpMV kernels s = A p^ + (r0,s) and y = A q^ +
    (q,y), (y,y): 3 + 2 (folded, Algorithm 7: 19 per iteration) or 3 + 3
    (Algorithm 10: 23 per iteration).  CA-BiCGStab (Algorithm 8, folded), its
    two SpMV kernels z = A s + (q,y), (y,y) (reads s, r, w, writes z: 4) and
    w = A r + five dots (reads r, r0, s, z, writes w: 5), and the two update
    kernels p, s (reads r, p, s, w, z, writes p, s: 7) and x, r (reads r, s,
    w, z, x, p, writes x, r: 8): 24 per iteration.
    """
    vec = 8 * N
    mat = 0 if stencil else (4 * N + 8 * dia * N if dia else 4 * (N + 1) + (8 + index_bytes) * nnz)
    if dia and codes:
        mat = 8 * N + 16 * 8 * dia
    if variant == "ca_bicgstab":
        return mat + 4 * vec, mat + 5 * vec, 24 * vec + 2 * mat
    if variant == "bicgstab":
        if folded:
            return mat + 3 * vec, mat + 2 * vec, 19 * vec + 2 * mat
        return mat + 3 * vec, mat + 3 * vec, 23 * vec + 2 * mat
    if folded:
        return mat + 10 * vec, mat + 12 * vec, 22 * vec + 2 * mat
    return mat + 16 * vec, mat + 18 * vec, 34 * vec + 2 * mat


def grid_coefficients(rp, col, val, n: int, N: int):
    """Per-row coefficients of an assembled 3-D 27-point CSR matrix on the n^3
    grid, term-major as pbcgs_op_stencil takes them (term (dz, dy, dx) of row r
    at term * N + r, dz slowest); slots of terms that leave the grid are NaN."""
    import torch
    rows = torch.repeat_interleave(torch.arange(N, device=rp.device), (rp[1:] - rp[:-1]).to(torch.int64))
    off = col.to(torch.int64) - rows
    n2 = n * n
    dz = torch.div(off + n2 // 2, n2, rounding_mode="floor")
    rem = off - dz * n2
    dy = torch.div(rem + n // 2, n, rounding_mode="floor")
    dx = rem - dy * n
    term = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)
    coef = torch.full((27 * N,), float("nan"), dtype=torch.float64, device=rp.device)
    coef[term * N + rows] = val
    del rows, off, dz, rem, dy, dx, term
    return coef


def algorithmic_bytes_mf27(n: int, variant: str):
    """Algorithmic HBM bytes (K_a, K_b, iteration) of the folded solvers on the
    matrix-free 27-point operator of an n^3 grid: each product reads the
    (n+1)^3 cell coefficients and gathers dinv (the column scaling of A M^{-1})
    besides its input vector; the vector passes are those of the folded CSR
    solve (:func:`algorithmic_bytes`)."""
    N = n ** 3
    mat = 8 * (n + 1) ** 3 + 8 * N
    vec = 8 * N
    if variant == "bicgstab":
        return mat + 3 * vec, mat + 2 * vec, 19 * vec + 2 * mat
    return mat + 10 * vec, mat + 12 * vec, 22 * vec + 2 * mat


def fixed_iterations(solve_fn, m: int, warm: int = 3, reps: int = 5):
    """Device time of m iterations at tol = 0: ``solve_fn(maxit)`` runs one
    solve and returns its info (ms = HIP events from the setup to the last
    kernel).  Median of ``reps`` solves after ``warm`` warm-ups, minus the
    median of as many setup-only solves (maxit = 0), so only the iteration loop
    is counted."""
    for _ in range(warm):
        solve_fn(m)
    infos = [solve_fn(m) for _ in range(reps)]
    full = sorted(i.ms for i in infos)[reps // 2]
    setup = sorted(solve_fn(0).ms for _ in range(reps))[reps // 2]
    return {"us_per_iter": round((full - setup) / m * 1e3, 2), "setup_us": round(setup * 1e3, 1), "iters": m,
            "codes": bool(getattr(infos[-1], "value_codes", False))}


def algorithmic_bytes_cg(N: int, nnz: int, variant: str, jacobi: bool, index_bytes: int = 4, dia: int = 0,
                         codes: bool = False):
    """Algorithmic HBM bytes of one iteration of the CG family (Section 2) on
    a CSR operator with Jacobi by a constant (a scalar, no vector) or none.

    CG (Algorithm 2): s = A p (gathers p, writes s), x/r/u (reads p, x, r, s,
    writes x, r and u), p (reads u, p, writes p): 12 vector passes with
    Jacobi, 11 without (u = r).  Chronopoulos & Gear (Algorithm 4): p, s, x,
    r, u (reads u, p, w, s, x, r, writes p, s, x, r, u) and w = A u (gathers
    u, reads r, writes w): 14, or 11 without.  p-CG (Algorithm 6): one
    kernel reading m (gathered), w, z, q, s, u, p, x, r and writing z, q, s,
    p, x, r, u, w and the next m: 18; without a preconditioner q = s, u = r,
    m = w: 12.  One SpMV per iteration in each.
    """
    vec = 8 * N
    mat = 4 * N + 8 * dia * N if dia else 4 * (N + 1) + (8 + index_bytes) * nnz
    if dia and codes:
        mat = 8 * N + 16 * 8 * dia  # value-indexed layout (see algorithmic_bytes)
    passes = {"cg": (12, 11), "cgcg": (14, 11), "pipe_cg": (18, 12)}[variant][0 if jacobi else 1]
    return passes * vec + mat


def host_cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def run_cpu_child(args):
    """Times the oracle in a child process that loads no GPU library, with
    OpenMP threads bound close to the cores (OMP_PROC_BIND must be set before
    the OpenMP runtime starts, which the parent's torch import already did)."""
    import subprocess
    nproc = len(os.sched_getaffinity(0))
    # a preset OMP_NUM_THREADS (the host's CPU share) wins over the affinity mask
    threads = os.environ.get("OMP_NUM_THREADS") or str(nproc)
    env = dict(os.environ, OMP_NUM_THREADS=threads, OMP_PROC_BIND="close", OMP_PLACES="cores")
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-child", "--n", str(args.n),
           "--cpu-seconds", str(args.cpu_seconds)]
    r = subprocess.run(cmd, env=env, capture_output=True, text=True, timeout=600)
    if r.returncode != 0:
        sys.stderr.write(r.stderr[-4000:])
        raise RuntimeError(f"oracle timing process failed with status {r.returncode}")
    out = json.loads(r.stdout.strip().splitlines()[-1])
    quota = None
    try:
        with open("/sys/fs/cgroup/cpu.max") as f:
            q, per = f.read().split()[:2]
            quota = None if q == "max" else round(int(q) / int(per), 2)
    except (OSError, ValueError):
        pass
    out["host"].update({"nproc": nproc, "cgroup_cpu_quota": quota, "omp_num_threads": int(threads)})
    return out


def cpu_child(args):
    """The oracle (plain C, -O3, OpenMP) on the benchmark system: per-iteration
    cost in the fixed-iteration mode (tol = 0, slope between two iteration
    counts, so the setup and the fold of A M^-1 cancel; median of 3) with all
    cores and with one thread, one complete solve at tol 1e-8, and SciPy's
    bicgstab as a sanity line.  Prints one JSON object."""
    import numpy as np

    import oracle
    from paper_1612_01395_amd import inputs

    w = inputs.workload("c2", n=args.n)
    Ah = oracle.assemble_workload(w)
    bh = oracle.spmv(Ah, inputs.x_true(w.N))
    dinv = oracle.jacobi_dinv(Ah)
    ncores = oracle.get_threads()

    def solve_s(m, tol=0.0):
        t0 = time.perf_counter()
        _, inf = oracle.solve_folded(Ah, bh, algo=oracle.ALG_PBICGSTAB_RR, dinv=dinv, tol=tol, maxit=m,
                                     rr_period=w.rr_period)
        return time.perf_counter() - t0, inf

    def per_iter(m1, m2, threads):
        oracle.set_threads(threads)
        t1 = sorted(solve_s(m1)[0] for _ in range(3))[1]
        t2 = sorted(solve_s(m2)[0] for _ in range(3))[1]
        return (t2 - t1) / (m2 - m1)

    t_start = time.perf_counter()
    s_all = per_iter(10, 40, ncores)
    s_one = per_iter(4, 12, 1)
    oracle.set_threads(ncores)
    tts, inf = solve_s(w.maxit, w.tol)
    # SciPy's BiCGStab (a library Algorithm 7, one process) on the same system, 20 iterations
    import scipy.sparse.linalg as spla
    As = Ah.to_scipy()
    its = [0]

    def cb(_):
        its[0] += 1

    t0 = time.perf_counter()
    spla.bicgstab(As, bh, rtol=1e-30, maxiter=20, callback=cb)
    s_scipy = (time.perf_counter() - t0) / max(its[0], 1)
    wall = time.perf_counter() - t_start
    print(json.dumps({
        "value": round(1.0 / s_all, 3), "unit": "iters/s", "cores": ncores, "kind": "oracle",
        "sample": f"the {w.n}^3 benchmark system, folded-Jacobi p-BiCGStab+RR, tol 0: seconds per iteration from "
                  f"the slope between 10 and 40 iterations (median of 3 each) with {ncores} OpenMP threads "
                  f"(one thread: 4 and 12 iterations); "
                  f"{wall:.1f} s of CPU work in all (with the lines below)",
        "host": {"cpu_model": host_cpu_model(),
                 "omp_proc_bind": os.environ.get("OMP_PROC_BIND", ""), "oracle_build": "gcc -O3 -fopenmp -ffp-contract=off"},
        "one_thread_iters_per_s": round(1.0 / s_one, 3),
        "parallel_speedup": round(s_one / s_all, 2),
        "time_to_solution_s": round(tts, 3), "iterations_to_tol": inf["iters"],
        "scipy_bicgstab_iters_per_s": round(1.0 / s_scipy, 3),
    }), flush=True)


def main():
    args = parse()
    if args.cpu_child:
        cpu_child(args)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the library has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1612_01395_amd import inputs, solver

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    w = inputs.workload("c2", n=args.n)
    N = w.N
    legs = set(args.only.split(",")) if args.only else {"pipe", "index32", "bicg", "explicit", "stencil", "fixed", "cg",
                                                         "precision", "batched", "sweep", "paper", "configs"}

    # ---- inputs resident in HBM -------------------------------------------------
    rp, col, val = solver.assemble_convdiff(w.dim, w.n, w.npts, w.beta)
    nnz = val.numel()
    A = solver.csr(rp, col, val)
    ib = A.index_bytes  # 2: the operator holds the compact int16 column copy
    nd = A.diagonals    # 7: the solves read the operator through its diagonal layout
    xt = torch.from_numpy(inputs.x_true(N)).to(dev)
    b = solver.spmv(A, xt)
    mid = w.n // 2
    crow = mid + w.n * mid + w.n * w.n * mid  # an interior row: all 7 coefficients
    coef = val[rp[crow].item(): rp[crow + 1].item()].cpu().tolist()
    S = solver.stencil(w.n, w.n, w.n, coef) if len(coef) == 7 else None
    xbuf = torch.empty_like(b)
    torch.cuda.synchronize()

    common = dict(tol=w.tol, maxit=w.maxit, rr_period=w.rr_period)
    # launch shapes from the autotuner (never change a result), kept on the
    # operator per variant and read path and in the library's launch-shape
    # cache: each leg is tuned for its own variant and preconditioner form
    # before it is timed, unless the cache file already holds its shape
    shapes = {}
    shape_source = {}
    if args.tune_cache:
        try:
            n_loaded = solver.load_tune_cache(args.tune_cache)
            progress(f"launch-shape cache {args.tune_cache}: {n_loaded} entries")
        except (OSError, ValueError) as e:
            progress(f"launch-shape cache {args.tune_cache} not read: {e}")

    def tune_for(op, variant, precond, label, **extra):
        cached = None if args.retune else solver.tuned_shape(
            op, variant, extra.get("precision", "fp64"), extra.get("index32", False),
            extra.get("diagonal_layout", True))
        if cached is not None:
            shapes[label] = cached
            shape_source[label] = "cache"
            return {"best": cached}
        rep_ = solver.tune(op, b, iters=40, variant=variant, precond=precond, rr_period=w.rr_period, **extra)
        shapes[label] = rep_["best"]
        shape_source[label] = "measured"
        if args.tune_cache:
            try:
                solver.save_tune_cache(args.tune_cache)
            except OSError as e:
                progress(f"launch-shape cache {args.tune_cache} not written: {e}")
        return rep_

    tune = tune_for(A, "pbicgstab_rr", "jacobi_folded", "pipe")

    def timed_leg(op, variant, precond, label, **extra):
        tune_for(op, variant, precond, label, **extra)
        for _ in range(args.warmup):
            solver.solve(op, b, variant=variant, precond=precond, out=xbuf, **common, **extra)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        iters = 0
        last = None
        for _ in range(args.steps):
            _, info = solver.solve(op, b, variant=variant, precond=precond, out=xbuf, **common, **extra)
            iters += info.iters
            last = info
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        return iters, dt, last

    # legs: (operator, variant, preconditioner form)
    LEGS = {
        "pipe": ("csr", "pbicgstab_rr", "jacobi_folded"),        # the metric
        "bicg": ("csr", "bicgstab", "jacobi_folded"),
        "ca": ("csr", "ca_bicgstab", "jacobi_folded"),
        "pipe_norr": ("csr", "pbicgstab", "jacobi_folded"),
        "pipe_i32": ("csr", "pbicgstab_rr", "jacobi_folded", {"index32": True}),  # int32 columns
        "pipe_csr": ("csr", "pbicgstab_rr", "jacobi_folded", {"diagonal_layout": False}),  # CSR stream, compact columns
        "pipe_alg11": ("csr", "pbicgstab_rr", "jacobi"),
        "bicg_alg10": ("csr", "bicgstab", "jacobi"),
        "st_pipe": ("stencil", "pbicgstab_rr", "jacobi_folded"),
        "st_bicg": ("stencil", "bicgstab", "jacobi_folded"),
    }
    groups = {"pipe": ["pipe", "pipe_norr"], "index32": ["pipe_i32", "pipe_csr"], "bicg": ["bicg", "ca"], "explicit": ["pipe_alg11", "bicg_alg10"],
              "stencil": ["st_pipe", "st_bicg"]}
    res = {}
    for g in ("pipe", "index32", "bicg", "explicit", "stencil"):
        if g not in legs:
            continue
        for leg in groups[g]:
            kind, variant, precond, *extra = LEGS[leg]
            op = A if kind == "csr" else S
            if op is None:
                continue
            res[leg] = timed_leg(op, variant, precond, leg, **(extra[0] if extra else {}))
            progress(f"leg {leg} done")
    # the fixed-iteration legs and the per-kernel roofline run the folded solves at their tuned shapes
    tune = tune_for(A, "pbicgstab_rr", "jacobi_folded", "pipe")
    tune_for(A, "bicgstab", "jacobi_folded", "bicg")
    tune_for(A, "ca_bicgstab", "jacobi_folded", "ca")
    if S is not None:
        tune_for(S, "pbicgstab_rr", "jacobi_folded", "st_pipe")
        tune_for(S, "bicgstab", "jacobi_folded", "st_bicg")

    progress("section: fixed-iteration mode")
    # ---- fixed-iteration mode: tol = 0, 200 iterations, device-timed -----------
    fixed = {}
    if "fixed" in legs:
        fixed = {"mode": "tol = 0, a fixed number of iterations (200 for the 128^3, 2-D and batched systems, 50 for "
                         "the 256^3 ones), HIP events from the setup to the last kernel minus a setup-only solve, "
                         "median of 5 after 3 warm-ups; folded Jacobi where the configuration has Jacobi"}
        c2f = {}
        for key, op_, variant in (("pbicgstab_rr_csr", A, "pbicgstab_rr"), ("bicgstab_csr", A, "bicgstab"),
                                  ("ca_bicgstab_csr", A, "ca_bicgstab"), ("pbicgstab_rr_stencil", S, "pbicgstab_rr"),
                                  ("bicgstab_stencil", S, "bicgstab")):
            if op_ is None:
                continue
            r = fixed_iterations(lambda m, op_=op_, variant=variant: solver.solve(
                op_, b, variant=variant, precond="jacobi_folded", tol=0.0, maxit=m, rr_period=w.rr_period,
                out=xbuf)[1], 200)
            _, _, pib = algorithmic_bytes(N, nnz, variant, op_ is S, index_bytes=ib, dia=nd, codes=r.pop("codes"))
            r["gbps_effective"] = round(pib / (r["us_per_iter"] * 1e-6) / 1e9, 1)
            c2f[key] = r
        c2f["pbicgstab_over_bicgstab_csr"] = round(c2f["bicgstab_csr"]["us_per_iter"]
                                                   / c2f["pbicgstab_rr_csr"]["us_per_iter"], 4)
        fixed[f"c2_{args.n}"] = c2f
        # latency-bound sizes: the marginal cost of an iteration (slope between
        # 50 and 200 iterations) and the fixed cost of a solve (intercept)
        for wname, side, pc in (("c1", 64, None), ("c2", 32, "jacobi_folded")):
            ws = inputs.workload(wname, n=side)
            rps, cols, vals = solver.assemble_convdiff(ws.dim, ws.n, ws.npts, ws.beta)
            As = solver.csr(rps, cols, vals)
            bs = solver.spmv(As, torch.from_numpy(inputs.x_true(ws.N)).to(dev))
            xs = torch.empty_like(bs)
            entry = {}
            for variant in ("pbicgstab_rr", "bicgstab"):
                med = {}
                for m in (50, 200):
                    kw = dict(variant=variant, precond=pc, tol=0.0, maxit=m, rr_period=ws.rr_period, out=xs)
                    solver.solve(As, bs, **kw)
                    times = sorted(solver.solve(As, bs, **kw)[1].ms for _ in range(9))
                    med[m] = times[4] * 1e3
                slope = (med[200] - med[50]) / 150.0
                entry[variant] = {"marginal_us_per_iter": round(slope, 2),
                                  "fixed_us_per_solve": round(med[50] - 50 * slope, 1)}
            entry["ratio_marginal"] = round(entry["bicgstab"]["marginal_us_per_iter"]
                                            / entry["pbicgstab_rr"]["marginal_us_per_iter"], 3)
            fixed[f"{wname}_{side}"] = entry
            del As, bs, xs, rps, cols, vals

    progress("section: the CG family")
    # ---- the CG family (Section 2) on the symmetric counterpart of the operator --
    cgfam = None
    if "cg" in legs:
        cgfam = {"workload": "3-D 7-point Poisson (beta = 0), CSR FP64, Jacobi, tol 1e-8; one step = one full "
                             "solve; at the benchmark grid and at 32^3 (latency-bound)"}
        for side in (args.n, 32):
            ws = inputs.workload("c2s", n=side)
            rps, cols, vals = solver.assemble_convdiff(ws.dim, ws.n, ws.npts, ws.beta)
            As = solver.csr(rps, cols, vals)
            bs = solver.spmv(As, torch.from_numpy(inputs.x_true(ws.N)).to(dev))
            xs = torch.empty_like(bs)
            torch.cuda.synchronize()
            entry = {}
            for variant in ("cg", "cgcg", "pipe_cg"):
                kw = dict(variant=variant, precond="jacobi", tol=ws.tol, maxit=ws.maxit, out=xs)
                for _ in range(args.warmup):
                    solver.solve(As, bs, **kw)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                its = 0
                for _ in range(args.steps):
                    _, cinfo = solver.solve(As, bs, **kw)
                    its += cinfo.iters
                torch.cuda.synchronize()
                cdt = time.perf_counter() - t0
                rate = its / cdt
                entry[variant] = {"iters_per_s": round(rate, 2), "iters_per_solve": cinfo.iters,
                                  "ms_per_solve": round(cdt / args.steps * 1e3, 3),
                                  "gbps_effective": round(algorithmic_bytes_cg(ws.N, vals.numel(), variant, True,
                                                                              As.index_bytes, As.diagonals,
                                                                              cinfo.value_codes)
                                                          * rate / 1e9, 1),
                                  "syncs_per_iter": cinfo.syncs_per_iter, "relres_true": cinfo.relres_true}
            cgfam[f"{side}^3"] = entry
            del As, bs, xs, rps, cols, vals

    progress("section: roofline of the dominant kernel")
    # ---- roofline of the dominant kernel: one solve with per-kernel events -------
    _, pinfo = solver.solve(A, b, variant="pbicgstab_rr", precond="jacobi_folded", out=xbuf, time_kernels=True,
                            **common)
    ba, bb, _ = algorithmic_bytes(N, nnz, "pbicgstab", False, index_bytes=ib, dia=nd, codes=pinfo.value_codes)
    avg = [pinfo.kernel_ms[k] / max(pinfo.kernel_calls[k], 1) for k in range(2)]
    dom = 0 if pinfo.kernel_ms[0] >= pinfo.kernel_ms[1] else 1
    dom_bytes = (ba, bb)[dom]
    achieved = dom_bytes / (avg[dom] * 1e-3) / 1e9
    # the launch grid at the tuned shape: ceil(N / (256 R)) workgroups of 256 threads
    grid_threads = -(-N // (256 * tune["best"])) * 256
    roofline = {
        "bound": "hbm",
        "kernel": ("k_pa (t = A w, recurrences, (q,y),(y,y))", "k_pb (v = A z, x/r/w updates, 5 dots)")[dom],
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": measured_traffic(("k_pa", "k_pb")[dom], grid_threads),
        "bytes_per_launch": dom_bytes,
        "grid_threads": grid_threads,
        "rows_per_wave_blocks": tune["best"],
        "column_index_bytes": ib,
        "operator_layout": (f"diagonal layout, {nd} diagonals, value-indexed (an 8-byte word of one-byte codes "
                            f"per row, a 16-entry value table per diagonal)" if pinfo.value_codes else
                            f"diagonal layout, {nd} diagonals (4-byte row mask + 8 bytes per diagonal and row)")
        if nd else f"CSR stream, {ib}-byte column indices",
        "avg_launch_us": round(avg[dom] * 1e3, 2),
        "other_kernel_avg_us": round(avg[1 - dom] * 1e3, 2),
        "launches_timed": pinfo.kernel_calls[dom],
        # the two fused kernels take nearly the same time, so which one is
        # dominant can change from run to run: both, side by side
        "per_kernel": {name: {"avg_launch_us": round(avg[k] * 1e3, 2), "bytes_per_launch": (ba, bb)[k],
                              "achieved": round((ba, bb)[k] / (avg[k] * 1e-3) / 1e9, 1),
                              "frac": round((ba, bb)[k] / (avg[k] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                              "traffic": measured_traffic(name, grid_threads)}
                       for k, name in enumerate(("k_pa", "k_pb"))},
    }

    progress("section: precision form at 256^3")
    # ---- precision form at 256^3 (tol 1e-10): binary32 + binary64 replacement vs binary64
    precision = None
    if "precision" in legs:
        w4 = inputs.workload("c4")
        rp4, col4, val4 = solver.assemble_convdiff(w4.dim, w4.n, w4.npts, w4.beta)
        A4 = solver.csr(rp4, col4, val4)
        b4 = solver.spmv(A4, torch.from_numpy(inputs.x_true(w4.N)).to(dev))
        x4 = torch.empty_like(b4)

        def leg4(prec, k):
            kw = dict(variant="pbicgstab_rr", precond="jacobi_folded", tol=w4.tol, maxit=w4.maxit, rr_period=k,
                      precision=prec, out=x4)
            solver.solve(A4, b4, **kw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            its = 0
            for _ in range(3):
                _, inf = solver.solve(A4, b4, **kw)
                its += inf.iters
            torch.cuda.synchronize()
            dt4 = (time.perf_counter() - t0) / 3
            return {"iters_per_s": round(its / 3 / dt4, 1), "iters_per_solve": inf.iters, "n_rr": inf.n_rr,
                    "rr_period": k, "ms_per_solve": round(dt4 * 1e3, 2), "relres_true": inf.relres_true,
                    "status": inf.status}

        f64 = leg4("fp64", 50)
        x64 = x4.clone()
        f32 = leg4("fp32_rr64", w4.rr_period)
        f32["err_vs_fp64_solution"] = (torch.linalg.norm(x4 - x64) / torch.linalg.norm(x64)).item()
        if "fixed" in legs:
            c4f = {}
            for prec, k in (("fp64", 50), ("fp32_rr64", w4.rr_period)):
                c4f[prec] = fixed_iterations(lambda m, prec=prec, k=k: solver.solve(
                    A4, b4, variant="pbicgstab_rr", precond="jacobi_folded", tol=0.0, maxit=m, rr_period=k,
                    precision=prec, out=x4)[1], 50)
                c4f[prec]["rr_period"] = k
            c4f["fp32_over_fp64_per_iter"] = round(c4f["fp64"]["us_per_iter"] / c4f["fp32_rr64"]["us_per_iter"], 4)
            fixed[f"c4_{w4.n}"] = c4f
        precision = {"workload": f"3-D 7-point {w4.n}^3 (N={w4.N}, nnz={val4.numel()}), folded Jacobi, "
                                 f"tol {w4.tol:g}; the binary64 solve equals the oracle's bit for bit",
                     "fp64": f64, "fp32_rr64": f32,
                     "time_to_solution_speedup": round(f64["ms_per_solve"] / f32["ms_per_solve"], 4)}
        del A4, rp4, col4, val4, b4, x4, x64
        torch.cuda.empty_cache()

    progress("section: the other configurations")
    # ---- the other configurations: 2-D 64^2 (latency-bound) and 3-D 27-point 256^3, assembled (matrix-bound)
    # and matrix-free
    other_cfg = None
    if "configs" in legs:
        other_cfg = {}

        def solve_leg(op, rhs, xo, variant, precond, wc, steps, **extra):
            kwc = dict(variant=variant, precond=precond, tol=wc.tol, maxit=wc.maxit, rr_period=wc.rr_period, out=xo,
                       **extra)
            solver.solve(op, rhs, **kwc)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            its = 0
            for _ in range(steps):
                _, inf = solver.solve(op, rhs, **kwc)
                its += inf.iters
            torch.cuda.synchronize()
            dtc = time.perf_counter() - t0
            return {"iters_per_s": round(its / dtc, 1), "us_per_iter": round(dtc / its * 1e6, 2),
                    "iters_per_solve": inf.iters, "ms_per_solve": round(dtc / steps * 1e3, 3),
                    "syncs_per_iter": inf.syncs_per_iter, "relres_true": inf.relres_true}

        for name, precond, steps in (("c1", None, 20), ("c3", "jacobi_folded", 2)):
            if name not in args.configs.split(","):
                continue
            wc = inputs.workload(name)
            kappa = None
            if wc.npts == 27:
                kappa = torch.from_numpy(inputs.kappa_cells(wc.n, wc.kappa_sigma)).to(dev)
            rpc, colc, valc = solver.assemble_convdiff(wc.dim, wc.n, wc.npts, wc.beta, kappa, wc.shift)
            Ac = solver.csr(rpc, colc, valc)
            bc = solver.spmv(Ac, torch.from_numpy(inputs.x_true(wc.N)).to(dev))
            xc = torch.empty_like(bc)
            row = {"workload": f"{wc.dim}-D {wc.npts}-point {wc.n}^{wc.dim} (N={wc.N}, nnz={valc.numel()}), "
                               f"precond {precond or 'none'}, tol {wc.tol:g}, RR every {wc.rr_period}"}
            row["operator_layout"] = (f"diagonal layout, {Ac.diagonals} diagonals" if Ac.diagonals
                                      else f"CSR stream, {Ac.column_form} columns")
            for variant in ("pbicgstab_rr", "bicgstab"):
                row[variant] = solve_leg(Ac, bc, xc, variant, precond, wc, steps)
            row["pbicgstab_over_bicgstab_iters_per_s"] = round(
                row["pbicgstab_rr"]["iters_per_s"] / row["bicgstab"]["iters_per_s"], 4)
            if Ac.diagonals and name == "c3":
                row["csr_stream"] = {"operator": f"CSR stream, {Ac.column_form} columns"}
                for variant in ("pbicgstab_rr", "bicgstab"):
                    row["csr_stream"][variant] = solve_leg(Ac, bc, xc, variant, precond, wc, steps,
                                                           diagonal_layout=False)
            if name == "c3":
                # the same operator matrix-free: entries formed from the cell coefficients (bitwise the CSR results)
                M27 = solver.convdiff27(wc.n, kappa, wc.beta, wc.shift)
                mf = {"operator": "matrix-free 27-point (pbcgs_op_convdiff27), folded Jacobi, "
                                  "8 bytes of kappa per row and product instead of the CSR matrix"}
                for variant in ("pbicgstab_rr", "bicgstab"):
                    mf[variant] = solve_leg(M27, bc, xc, variant, precond, wc, steps)
                mf["pbicgstab_over_bicgstab_iters_per_s"] = round(
                    mf["pbicgstab_rr"]["iters_per_s"] / mf["bicgstab"]["iters_per_s"], 4)
                mf["over_csr_iters_per_s"] = round(mf["pbicgstab_rr"]["iters_per_s"]
                                                   / row["pbicgstab_rr"]["iters_per_s"], 4)
                # per-kernel figures of the fused kernels on the matrix-free operator
                _, kinfo = solver.solve(M27, bc, variant="pbicgstab_rr", precond=precond, tol=wc.tol,
                                        maxit=wc.maxit, rr_period=wc.rr_period, out=xc, time_kernels=True)
                mba, mbb, _ = algorithmic_bytes_mf27(wc.n, "pbicgstab")
                mf["kernels"] = {}
                for kk, kname in enumerate(("k_pa", "k_pb")):
                    kus = kinfo.kernel_ms[kk] / max(kinfo.kernel_calls[kk], 1) * 1e3
                    kb_ = (mba, mbb)[kk]
                    mf["kernels"][kname] = {"avg_launch_us": round(kus, 2), "bytes_per_launch": kb_,
                                            "achieved_gbps": round(kb_ / (kus * 1e-6) / 1e9, 1),
                                            "frac": round(kb_ / (kus * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)}
                row["matrix_free"] = mf
                # the same operator as a stencil with per-row coefficients: the assembled
                # values rearranged term-major (term (dz, dy, dx) of row r at term * N + r)
                G27 = grid_coefficients(rpc, colc, valc, wc.n, wc.N)
                S27 = solver.stencil(wc.n, wc.n, wc.n, G27, npts=27)
                pr = {"operator": "27-point stencil with per-row coefficients (pbcgs_op_stencil, coef_per_row = 1), "
                                  "216 bytes of coefficients per row and product"}
                for variant in ("pbicgstab_rr", "bicgstab"):
                    pr[variant] = solve_leg(S27, bc, xc, variant, precond, wc, steps)
                xs27 = xc.clone()
                solver.solve(Ac, bc, variant="bicgstab", precond=precond, tol=wc.tol, maxit=wc.maxit,
                             rr_period=wc.rr_period, out=xc)
                pr["solution_bitwise_equal_to_assembled"] = bool(torch.equal(xs27, xc))
                del xs27
                row["per_row_stencil"] = pr
                if "fixed" in legs:
                    c3f = {}
                    for key, op_, variant, lay in (
                            ("pbicgstab_rr_assembled", Ac, "pbicgstab_rr", True), ("bicgstab_assembled", Ac, "bicgstab", True),
                            ("pbicgstab_rr_csr_stream", Ac, "pbicgstab_rr", False),
                            ("bicgstab_csr_stream", Ac, "bicgstab", False),
                            ("pbicgstab_rr_matrix_free", M27, "pbicgstab_rr", True),
                            ("bicgstab_matrix_free", M27, "bicgstab", True),
                            ("pbicgstab_rr_per_row_stencil", S27, "pbicgstab_rr", True),
                            ("bicgstab_per_row_stencil", S27, "bicgstab", True)):
                        c3f[key] = fixed_iterations(lambda m, op_=op_, variant=variant, lay=lay: solver.solve(
                            op_, bc, variant=variant, precond=precond, tol=0.0, maxit=m, rr_period=wc.rr_period,
                            out=xc, diagonal_layout=lay)[1], 50)
                    fixed[f"c3_{wc.n}"] = c3f
                del M27, S27, G27
            other_cfg[name] = row
            del Ac, rpc, colc, valc, bc, xc, kappa
            torch.cuda.empty_cache()

    progress("section: the paper's test problems")
    # ---- the paper's test problems (Section 5): 1000^2 five-point stencils, x_hat = 1, tol 1e-6
    paper = None
    if "paper" in legs:
        eps = 1.0 - 0.001
        paper = {}
        for name, coef, variants in (("PTP1", [-eps, -1.0, 4.0, -eps, -1.0], ("bicgstab", "pbicgstab", "pbicgstab_rr")),
                                     ("PTP2", [-1.0, -1.0, 1.0, -1.0, -1.0], ("bicgstab", "pbicgstab"))):
            Sp = solver.stencil(1000, 1000, 1, coef)
            bp = solver.spmv(Sp, torch.ones(1000 * 1000, dtype=torch.float64, device=dev))
            xp = torch.empty_like(bp)
            row = {}
            for variant in variants:
                kwp = dict(variant=variant, tol=1e-6, maxit=4000, rr_period=100, rr_max=10, out=xp)
                solver.solve(Sp, bp, **kwp)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, inf = solver.solve(Sp, bp, **kwp)
                torch.cuda.synchronize()
                row[variant] = {"iterations": inf.iters, "ms": round((time.perf_counter() - t0) * 1e3, 2),
                                "true_residual": inf.relres_true * torch.linalg.norm(bp).item()}
            paper[name] = row
        paper["note"] = ("paper (20 nodes, 240 ranks): PTP1 205-282 iterations, PTP2 1283-2112; "
                         "matrix-free stencil here, bitwise equal to the CSR solve and the oracle")

    progress("section: size sweep")
    # ---- size sweep: where the two kernel boundaries per iteration pay off
    sweep = None
    if "sweep" in legs:
        sweep = {}
        for ns in (16, 24, 32, 48, 64, 96):
            ws_ = inputs.workload("c2", n=ns)
            rps, cols, vals = solver.assemble_convdiff(ws_.dim, ns, ws_.npts, ws_.beta)
            As = solver.csr(rps, cols, vals)
            bs_ = solver.spmv(As, torch.from_numpy(inputs.x_true(ws_.N)).to(dev))
            xs_ = torch.empty_like(bs_)
            row = {}
            for variant in ("pbicgstab_rr", "bicgstab"):
                kws = dict(variant=variant, precond="jacobi_folded", tol=ws_.tol, maxit=ws_.maxit,
                           rr_period=ws_.rr_period, out=xs_)
                solver.solve(As, bs_, **kws)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                its = 0
                for _ in range(5):
                    _, inf = solver.solve(As, bs_, **kws)
                    its += inf.iters
                torch.cuda.synchronize()
                dts = time.perf_counter() - t0
                row[variant] = {"iters_per_s": round(its / dts, 1), "us_per_iter": round(dts / its * 1e6, 2),
                                "iters_per_solve": inf.iters}
            row["pbicgstab_over_bicgstab_iters_per_s"] = round(
                row["pbicgstab_rr"]["iters_per_s"] / row["bicgstab"]["iters_per_s"], 4)
            sweep[f"{ns}^3"] = row

    progress("section: batched form")
    # ---- batched form: 512 independent 2-D systems of uneven size, forward and adjoint
    batched = None
    if "batched" in legs:
        systems = inputs.batch_systems()
        bops, bbs, bws, bN, bnnz = [], [], [], [], []
        for sy in systems:
            rpk, colk, valk = solver.assemble_convdiff(2, sy.n, 5, sy.beta)
            Ak = solver.csr(rpk, colk, valk)
            Nk = sy.n * sy.n
            bops.append(Ak)
            bbs.append(solver.spmv(Ak, torch.from_numpy(inputs.batch_x_true(sy.k, Nk)).to(dev)))
            bws.append(torch.from_numpy(inputs.batch_loss_weights(sy.k, Nk)).to(dev))
            bN.append(Nk)
            bnnz.append(valk.numel())
        bts = [solver.transpose(Ak) for Ak in bops]
        outs = [torch.empty_like(bk) for bk in bbs]
        kwb = dict(tol=1e-8, maxit=20000, rr_period=50)
        # launch shape (per-system workgroup cap) from the autotuner, outside the timed
        # region, timed on complete solves: the systems stop at different iterations
        btune = solver.tune_batched(bops, bbs, iters=0, variant="pbicgstab_rr", **kwb)

        def batch_leg(ops_, rhs, variant, passes, diagonal_layout=True):
            kwl = dict(kwb, diagonal_layout=diagonal_layout)
            solver.solve_batched(ops_, rhs, variant=variant, outs=outs, **kwl)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            reps = 2
            for _ in range(reps):
                _, infs = solver.solve_batched(ops_, rhs, variant=variant, outs=outs, **kwl)
            torch.cuda.synchronize()
            dtb = (time.perf_counter() - t0) / reps
            its = [i.iters for i in infs]
            # the batch reads every system through its diagonal layout when all have
            # one, else int16 block offsets when every operator holds them
            nds = [op.diagonals for op in ops_]
            if diagonal_layout and all(nds):
                layout = "diagonal"
                mats = [4 * Nk + 8 * nd * Nk for Nk, nd in zip(bN, nds)]
            else:
                ibb = 2 if all(op.column_form == "block16" for op in ops_) else 4
                layout = f"csr, int{8 * ibb} columns"
                mats = [4 * (Nk + 1) + (8 + ibb) * zk for Nk, zk in zip(bN, bnnz)]
            byts = sum(it_ * (passes * 8 * Nk + 2 * mk) for it_, Nk, mk in zip(its, bN, mats))
            return {"ms_per_batch_solve": round(dtb * 1e3, 2), "operator_layout": layout,
                    "iters_total": int(sum(its)), "iters_max": int(max(its)),
                    "iters_per_s_aggregate": round(sum(its) / dtb, 1), "gbps_effective": round(byts / dtb / 1e9, 1),
                    "all_converged": all(i.status == 0 for i in infs),
                    "max_relres_true": max(i.relres_true for i in infs)}

        batched = {"workload": f"{len(systems)} 2-D 5-point systems, side log-uniform in [32, 512], "
                               f"beta ~ U[0,200]^2, sum N = {sum(bN)}, sum nnz = {sum(bnnz)}, CSR FP64, "
                               f"no preconditioner, tol 1e-8, RR every 50; one step = all systems solved",
                   "pbicgstab_rr": batch_leg(bops, bbs, "pbicgstab_rr", 22),
                   "bicgstab": batch_leg(bops, bbs, "bicgstab", 19),
                   "pbicgstab_rr_csr_stream": batch_leg(bops, bbs, "pbicgstab_rr", 22, diagonal_layout=False),
                   "adjoint_pbicgstab_rr": batch_leg(bts, bws, "pbicgstab_rr", 22),
                   "autotuned_workgroup_cap": btune["best"],
                   "autotuner_ms_per_batch_solve": {str(k): round(v, 1) for k, v in btune["tried"].items()}}
        batched["pbicgstab_over_bicgstab_time"] = round(
            batched["bicgstab"]["ms_per_batch_solve"] / batched["pbicgstab_rr"]["ms_per_batch_solve"], 4)
        if "fixed" in legs:
            c5f = {}
            for variant in ("pbicgstab_rr", "bicgstab"):
                c5f[variant] = fixed_iterations(lambda m, variant=variant: solver.solve_batched(
                    bops, bbs, variant=variant, outs=outs, tol=0.0, maxit=m, rr_period=50)[1][0], 200)
            c5f["note"] = "every one of the 512 systems runs the 200 iterations; us_per_iter is one iteration of all"
            fixed["c5_batch"] = c5f
        del bops, bbs, bws, bts, outs
        torch.cuda.empty_cache()

    if args.copy_calib:
        # a plain copy of known size: 256 MiB read + 256 MiB written per dispatch
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()

    progress("section: CPU baseline")
    # ---- CPU baseline: the oracle on a bounded sample, in a process of its own ---
    cpu = None
    if not args.no_cpu_baseline:
        cpu = run_cpu_child(args)

    it, dt, info = res.get("pipe", (0, 1.0, None))
    value = it / dt if it else None
    _, _, per_iter_bytes = algorithmic_bytes(N, nnz, "pbicgstab", False, index_bytes=ib, dia=nd,
                                             codes=bool(info and info.value_codes))
    out = {
        "metric": "p-BiCGStab iters/sec + HBM GB/s (3D 7-pt 128^3 FP64) vs plain BiCGStab, same GPU",
        "value": round(value, 2) if value else None,
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"3-D 7-point upwind convection-diffusion {w.n}^3 (N={N}, nnz={nnz}), "
                               f"beta=(50,30,10), CSR FP64, Jacobi (right preconditioning, A M^-1 formed), "
                               f"tol 1e-8, p-BiCGStab with residual replacement every {w.rr_period}; "
                               f"one step = one full solve",
                   "global_batch": 1, "parallelism": "single GPU"},
        "iters_per_solve": info.iters if info else None,
        "relres_true": info.relres_true if info else None,
        "gbps_effective": round(per_iter_bytes * value / 1e9, 1) if value else None,
        "syncs_per_iter": info.syncs_per_iter if info else None,
        "autotuned_rows_per_wave_blocks": tune["best"],
        "autotuned_rows_per_wave_blocks_per_leg": shapes,
        "launch_shape_source_per_leg": shape_source,
    }

    def leg_summary(key, variant, stencil, folded, index_bytes=ib, dia=nd):
        lit, ldt, linfo = res[key]
        lval = lit / ldt
        _, _, lbytes = algorithmic_bytes(N, nnz, variant, stencil, folded, index_bytes=index_bytes, dia=dia,
                                         codes=linfo.value_codes)
        return {"iters_per_s": round(lval, 2), "iters_per_solve": linfo.iters,
                "ms_per_solve": round(ldt / args.steps * 1e3, 3), "gbps_effective": round(lbytes * lval / 1e9, 1),
                "syncs_per_iter": linfo.syncs_per_iter, "relres_true": linfo.relres_true}

    if "bicg" in res:
        out["bicgstab"] = leg_summary("bicg", "bicgstab", False, True)
        if value:
            bval = out["bicgstab"]["iters_per_s"]
            out["pbicgstab_over_bicgstab_iters_per_s"] = round(value / bval, 4)
            out["pbicgstab_over_bicgstab_time_to_solution"] = round(
                out["bicgstab"]["ms_per_solve"] / (dt / args.steps * 1e3), 4)
    if "ca" in res:
        out["ca_bicgstab"] = leg_summary("ca", "ca_bicgstab", False, True)
        if value:
            out["pbicgstab_over_ca_bicgstab_iters_per_s"] = round(value / out["ca_bicgstab"]["iters_per_s"], 4)
    if "pipe_norr" in res:
        out["pbicgstab_without_replacement"] = leg_summary("pipe_norr", "pbicgstab", False, True)
    if "pipe_i32" in res:
        out["pbicgstab_rr_int32_columns"] = leg_summary("pipe_i32", "pbicgstab", False, True, index_bytes=4, dia=0)
        if value:
            out["diagonal_layout_over_int32_columns_iters_per_s"] = round(
                value / out["pbicgstab_rr_int32_columns"]["iters_per_s"], 4)
    if "pipe_csr" in res:
        out["pbicgstab_rr_csr_stream"] = leg_summary("pipe_csr", "pbicgstab", False, True, dia=0)
        if value:
            out["diagonal_layout_over_csr_stream_iters_per_s"] = round(
                value / out["pbicgstab_rr_csr_stream"]["iters_per_s"], 4)
    if "pipe_alg11" in res:
        out["explicit_jacobi"] = {"pbicgstab_rr_alg11": leg_summary("pipe_alg11", "pbicgstab", False, False),
                                  "bicgstab_alg10": leg_summary("bicg_alg10", "bicgstab", False, False)}
    for key, variant in (("st_pipe", "pbicgstab"), ("st_bicg", "bicgstab")):
        if key in res:
            out.setdefault("stencil", {})[variant] = leg_summary(key, variant, True, True)
    if fixed:
        out["fixed_iterations"] = fixed
    if cgfam is not None:
        out["cg_family"] = cgfam
    if precision is not None:
        out["precision_form"] = precision
    if batched is not None:
        out["batched"] = batched
    if sweep is not None:
        out["size_sweep_3d_7pt_csr_folded_jacobi"] = sweep
    if paper is not None:
        out["paper_test_problems"] = paper
    if other_cfg is not None:
        out["other_configs"] = other_cfg
    out["roofline"] = roofline
    out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
