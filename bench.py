"""Benchmark: BRAS-preconditioned CG time-to-solution vs Jacobi-PCG on one GPU.

One step = one complete BRAS-PCG solve (mass apply, BRAS apply and the CG
vector updates, every iteration, until the relative residual reaches the
workload's tolerance) on inputs already resident in device memory.  The
Jacobi-PCG solve of the same system, the BRAS apply bandwidth against the
HBM roofline and the CPU oracle (same workload, bounded sample) are reported
beside it.

Default workload: H(curl) Nedelec (first kind) degree 2 on 48^3 x 6 jittered
tetrahedra (4.27M DOFs), BRAS inverses stored in FP32 inside FP64 CG, tolerance
1e-8 (the tolerance the metric names).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
import argparse
import glob
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402

METRIC = "BRAS-PCG time to 1e-8 rel. residual vs Jacobi-PCG; BRAS apply HBM GB/s"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
BF16_PEAK_TFLOPS = 2500.0   # dense BF16 matrix-core peak (no sparsity)
DEFAULT = "n1curl2_3d_48_jit"


def algorithmic_bytes(w, n, E, n_loc, R, prec):
    """Bytes one BRAS apply must move (the unit of the roofline): x in and
    y out (float64), the map (int32 per broken DOF), the element data, and
    D^-1 when it is not folded into the stored inverses.  The broken
    intermediate and the transpose map are implementation traffic and are
    not counted."""
    nbr = E * n_loc
    vec = 8.0 * n * R
    if w.family in ("P", "B"):
        elem = 8.0 * E          # one coefficient per element (shared reference inverse)
        dinv = 8.0 * n
    else:
        esz = {"f64": 8, "f32": 4, "bf16": 2}[prec]
        elem = esz * E * n_loc * (n_loc + 1) / 2.0
        dinv = 0.0              # folded into the stored inverses
    return 2 * vec + 4.0 * nbr + elem + dinv


# sources of the operator passes and their data layout (the kernels the
# stored counter measurements describe): shared by every apply, then by form
COMMON_SOURCES = ("apply.hip", "cg_common.h", "block_reduce.h", "internal.h", "setup.hip")
FORM_SOURCES = {
    "patch": ("patch*.hip", "patch*.h", "patch_setup.cpp", "elem_lane.h"),   # one column, vector families
    "bf16": ("bf16.hip", "bf16_gram.h"),                                    # BF16 Gram-factor element pass
    "element": ("elem_lane.h", "lane_*.hip", "elem_mfma.hip"),              # element pass + reduce
}


def apply_form(w):
    """Which kernels a workload's BRAS apply runs (see FORM_SOURCES)."""
    if w.prec == "bf16":
        return "bf16"
    if w.nrhs == 1 and w.family not in ("P", "B"):
        return "patch"
    return "element"


def source_digest(w=None):
    """sha256 over the sources of the operator passes a workload's apply runs
    (all of them without a workload), to tell whether a stored counter
    measurement still describes the kernels being run."""
    pats = COMMON_SOURCES + (FORM_SOURCES[apply_form(w)] if w is not None
                             else tuple(p for v in FORM_SOURCES.values() for p in v))
    h = hashlib.sha256()
    files = set()
    for pat in pats:
        files.update(glob.glob(os.path.join(ROOT, "paper_2607_12138_amd", "csrc", pat)))
    for f in sorted(files):
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(workload):
    """HBM bytes per BRAS apply from the committed rocprofv3 counter summary
    of this workload, or None when the kernels changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "bras_apply_%s_traffic.json" % workload)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_digest") != source_digest(workloads.BY_NAME[workload]):
        return None
    return rec.get("hbm_bytes_per_apply")


def time_solves(prob, b, pc, tol, steps):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its = rel = st = None
    for _ in range(steps):
        x, st, its, rel = prob.solve(b, pc, rtol=tol)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps * 1e3, st, its, rel, x


def time_apply(fn, x, y, reps):
    """Average duration of fn on the current torch stream (the stream the
    library launches on), from HIP events around reps back-to-back calls."""
    import torch
    s = torch.cuda.current_stream()
    for _ in range(3):
        fn(x, y)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        fn(x, y)
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps * 1e3   # microseconds


def time_apply_cold(fn, x, y, reps, flush_bytes=1 << 29):
    """Average duration of fn with none of its data in the 256 MB Infinity
    Cache: a 512 MiB buffer is written on the same stream before each call,
    outside the HIP events that bracket the call."""
    import torch
    s = torch.cuda.current_stream()
    junk = torch.empty(flush_bytes // 8, dtype=torch.float64, device=x.device)
    fn(x, y)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for k in range(reps):
        junk.fill_(float(k))
        ev[k][0].record(s)
        fn(x, y)
        ev[k][1].record(s)
    torch.cuda.synchronize()
    return sum(a.elapsed_time(b) for a, b in ev) / reps * 1e3   # microseconds


def device_copy_gbs(reps=5):
    """Bytes read plus written per second by a plain 1 GiB device-to-device
    copy: the streaming rate HBM actually delivers, beside its 8 TB/s peak."""
    import torch
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        dst.copy_(src)
    e1.record(s)
    e1.synchronize()
    sec = e0.elapsed_time(e1) / reps * 1e-3
    del src, dst
    return 2 * (1 << 30) / sec / 1e9


def stationary_section(prob, b, w, steps):
    """Section 3's other solvers on the same system: damped fixed point with
    omega_bras = 2/(1 + lambda_max) and omega_diag = 1/lambda_max, and the
    Chebyshev semi-iteration on [1, 1.02 lambda_max] with BRAS (lambda_min >= 1,
    Cor. bras_lambda_min).  lambda_max by 200 power iterations from a seeded
    vector; as in the paper, its estimation is not part of the solve time."""
    import torch
    v0 = workloads.vector(prob.n, w.seed(4))
    lam_b = prob.lambda_max("bras", v0, 200)
    lam_d = prob.lambda_max("jacobi", v0, 200)
    runs = {
        "fixed_point_bras": lambda: prob.fixed_point(b, "bras", 2.0 / (1.0 + lam_b), rtol=w.tol),
        "fixed_point_jacobi": lambda: prob.fixed_point(b, "jacobi", 1.0 / lam_d, rtol=w.tol),
        "chebyshev_bras": lambda: prob.chebyshev(b, "bras", 1.0, 1.02 * lam_b, rtol=w.tol),
    }
    out = {"lambda_max_bras": round(lam_b, 6), "lambda_max_jacobi": round(lam_d, 6)}
    for name, fn in runs.items():
        fn()                                             # warm-up (graph capture)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            _, st, its, rel = fn()
        torch.cuda.synchronize()
        out[name] = {"ms": round((time.perf_counter() - t0) / steps * 1e3, 4), "iterations": int(max(its)),
                     "status": int(st), "relres": float(np.max(rel))}
    return out


def assembled_section(prob, x, y, bras_us, reps):
    """The assembled M_bras^-1 (CSR, float64 values, int32 columns) applied as a
    sparse product, against the matrix-free apply on the same input: the
    sparse form moves 12 bytes per stored entry, the element form the packed
    inverses once per element."""
    import torch
    from paper_2607_12138_amd import _lib as L
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    csr = prob.assemble(L.OP_BRAS)
    torch.cuda.synchronize()
    asm_s = time.perf_counter() - t0
    nnz = int(csr[1].numel())
    us = time_apply(lambda u, v: L.bras_csr_apply(prob.n, csr[0], csr[1], csr[2], u, v), x, y, reps)
    nbytes = 12 * nnz + 8 * (prob.n + 1) + 16 * prob.n
    del csr
    torch.cuda.empty_cache()
    return {"nnz": nnz, "assemble_s": round(asm_s, 3), "us_per_apply": round(us, 3), "bytes_per_apply": nbytes,
            "gbs": round(nbytes / (us * 1e-6) / 1e9, 1), "time_vs_matrix_free": round(us / bras_us, 3)}


def schur_section(prob, w, reps=3):
    """Section 4's sparse Schur-complement approximation -St = G M_bras^-1 G^T
    (eq. approx_positive_schur_general, C = 0) for a coupling G with one row per
    element holding its DOFs (the pattern of a discrete divergence or gradient
    on the cells) with seeded U[-1,1] values: the assembled BRAS operator, then
    the two device products (G M_bras^-1) G^T.  Best of reps, each from the
    assembled operator (its assembly is timed separately above)."""
    import torch
    from paper_2607_12138_amd import _lib as L
    from paper_2607_12138_amd.problem import spgemm, csr_transpose
    E, nl, n = prob.E, prob.n_loc, prob.n
    rp = torch.arange(0, (E + 1) * nl, nl, dtype=torch.int64, device="cuda")
    col = torch.from_numpy(np.ascontiguousarray(np.sort(prob.l2g, axis=1), dtype=np.int32).reshape(-1)).cuda()
    val = torch.from_numpy(workloads.vector(E * nl, w.seed(5))).cuda()
    G = (rp, col, val)
    B = prob.assemble(L.OP_BRAS)
    best, out = None, None
    try:
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            T = spgemm(G, B, E, n)
            Gt = csr_transpose(G, E, n)
            S = spgemm(T, Gt, E, n)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
            out = {"m": E, "n": n, "nnz_G": E * nl, "nnz_B": int(B[1].numel()), "nnz_T": int(T[1].numel()),
                   "nnz_St": int(S[1].numel())}
            del T, Gt, S
        out["ms"] = round(best * 1e3, 3)
    except L.BrasError as e:     # e.g. device memory for the sort of long rows: reported, not fatal to the bench
        out = {"error": str(e)}
    del B, G
    torch.cuda.empty_cache()
    return out


def cpu_baseline(w, its_gpu, budget_s=20.0, y_gpu=None):
    """The oracle's BRAS-PCG on the same workload, matrix-free (its element
    route), one thread.  Setup (mesh, numbering, element matrices and
    inverses) is excluded, as the paper excludes preconditioner
    construction.  A bounded sample: at most budget_s of iterations; the
    time per iteration is scaled to the GPU's iteration count.
    With y_gpu (the device BRAS apply of the right-hand side, column 0) it also
    returns that apply's error against the oracle's float64 one."""
    from threadpoolctl import threadpool_limits
    from oracle import fe, mesh, dofmap, assembly, pcg
    extra = {}
    with threadpool_limits(1):
        ref = fe.reference_element(w.family, w.dim, w.degree)
        coords, cells = mesh.structured_mesh(w.dim, w.N, jitter=w.jitter, seed=w.mesh_seed)
        rho = workloads.density(len(cells), w.seed(2)) if w.density else None
        pi, n, _ = dofmap.build_dofmap(cells, len(coords), ref.dofs_per_entity)
        mats = assembly.element_matrices(ref, coords, cells, rho)
        inv = assembly.element_inverses(mats)
        d = np.bincount(pi.ravel(), minlength=n).astype(float)
        b = workloads.rhs(n, w.nrhs, w.seed(1))
        b = b if b.ndim == 1 else np.ascontiguousarray(b[:, 0])   # column 0 of the device workload
        M = lambda v: assembly.mass_apply_matrix_free(pi, mats, v)        # noqa: E731
        C = lambda v: assembly.bras_apply_matrix_free(pi, inv, d, v)     # noqa: E731
        if y_gpu is not None:
            y64 = C(b)
            dy = y_gpu - y64
            extra = {"bras_apply_rel_err_2": float(np.linalg.norm(dy) / np.linalg.norm(y64)),
                     "bras_apply_rel_err_inf": float(np.max(np.abs(dy)) / np.max(np.abs(y64)))}
        t0 = time.perf_counter()
        M(b)
        C(b)
        est = time.perf_counter() - t0                  # about one iteration
        k = int(max(1, min(its_gpu, budget_s / max(est, 1e-6) - 1)))
        t0 = time.perf_counter()
        _, done, ok, _ = pcg.pcg(M, b, C, tol=w.tol, maxit=k)
        dt = time.perf_counter() - t0
    per_it = dt / max(done, 1)
    full = bool(ok)
    if full:
        extra["oracle_iterations"] = int(done)
    return extra, {
        "value": round(per_it * (done if full else its_gpu) * 1e3, 3),
        "unit": "ms per solve (BRAS-PCG, one right-hand side)",
        "cores": 1,
        "kind": "oracle",
        "sample": ("full solve, %d iterations" % done) if full else
                  ("%d of %d iterations of the oracle's matrix-free BRAS-PCG on column 0 of the same "
                   "workload (numpy, 1 thread; setup excluded), %.1f s, scaled to %d iterations"
                   % (done, its_gpu, dt, its_gpu)),
    }


def cpu_baseline_sampled(w, its_gpu, rows=None, y_rows=None, sample_elems=4096):
    """The cpu_baseline leg for workloads whose full oracle set-up (every
    element matrix and inverse in float64) does not fit a bounded CPU sample
    (the 32-column BF16 workload: 15 GB of element data).  Time: the oracle's
    matrix-free mass and BRAS applies over all 32 columns on the first
    sample_elems elements, scaled to all elements and to the device's
    iteration count (one mass and one BRAS apply per iteration).  Error: the
    oracle's float64 BRAS apply at the sampled DOFs `rows` (every element
    touching them included) against the device's values there, y_rows."""
    from threadpoolctl import threadpool_limits
    from oracle import fe, mesh, dofmap, assembly
    extra = {}
    with threadpool_limits(1):
        ref = fe.reference_element(w.family, w.dim, w.degree)
        coords, cells = mesh.structured_mesh(w.dim, w.N, jitter=w.jitter, seed=w.mesh_seed)
        rho = workloads.density(len(cells), w.seed(2)) if w.density else None
        pi, n, _ = dofmap.build_dofmap(cells, len(coords), ref.dofs_per_entity)
        d = np.bincount(pi.ravel(), minlength=n).astype(float)
        b = workloads.rhs(n, w.nrhs, w.seed(1))
        if rows is not None:
            sub = np.nonzero(np.isin(pi, rows).any(axis=1))[0]
            inv = assembly.element_inverses(assembly.element_matrices(ref, coords, cells[sub],
                                                                      None if rho is None else rho[sub]))
            y64 = assembly.bras_apply_matrix_free(pi[sub], inv, d, b)[rows]
            dy = y_rows - y64
            extra = {"bras_apply_rel_err_2": float(np.linalg.norm(dy) / np.linalg.norm(y64)),
                     "bras_apply_rel_err_inf": float(np.max(np.abs(dy)) / np.max(np.abs(y64))),
                     "error_sample": "%d DOFs x %d columns (the oracle's float64 apply at those DOFs, all %d "
                                     "elements touching them)" % (len(rows), w.nrhs, len(sub))}
        sub = np.arange(min(sample_elems, len(cells)))
        mats = assembly.element_matrices(ref, coords, cells[sub], None if rho is None else rho[sub])
        inv = assembly.element_inverses(mats)
        pis = pi[sub]
        t0 = time.perf_counter()
        reps = 0
        while True:
            for c in range(w.nrhs):
                assembly.mass_apply_matrix_free(pis, mats, b[:, c])
            assembly.bras_apply_matrix_free(pis, inv, d, b)
            reps += 1
            if time.perf_counter() - t0 > 10.0:
                break
        dt = (time.perf_counter() - t0) / reps
    per_it = dt * len(cells) / len(sub)
    return extra, {
        "value": round(per_it * its_gpu * 1e3, 3),
        "unit": "ms per solve of all %d right-hand sides" % w.nrhs,
        "cores": 1,
        "kind": "oracle",
        "sample": ("the oracle's matrix-free mass and BRAS applies of all %d columns on %d of %d elements "
                   "(numpy, 1 thread; set-up excluded), %d rounds in %.1f s, scaled to all elements and %d "
                   "iterations (vector updates not counted)" % (w.nrhs, len(sub), len(cells), reps, dt * reps,
                                                                 its_gpu)),
    }


def gradient_section(prob, w, b, steps=2):
    """x = M(rho)^-1 b and its gradient (autograd: BRAS-PCG forward, adjoint
    BRAS-PCG and the per-element contraction backward) for the density
    workload, loss 0.5 ||x - x*||^2, at the workload's tolerance."""
    import torch
    from paper_2607_12138_amd.autograd import mass_solve
    rho = torch.from_numpy(workloads.density(prob.E, w.seed(2))).cuda()
    xs = torch.from_numpy(workloads.target(prob.n, w.seed(3))).cuda()
    fw = bw = None
    for k in range(steps + 1):
        bt = b.clone().requires_grad_(True)
        rt = rho.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x = mass_solve(bt, rt, prob, w.tol)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss = 0.5 * torch.sum((x - xs) ** 2)
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if k > 0:   # the first pass captures the graphs
            fw = (t1 - t0) if fw is None else min(fw, t1 - t0)
            bw = (t2 - t1) if bw is None else min(bw, t2 - t1)
    return {"forward_ms": round(fw * 1e3, 3), "backward_ms": round(bw * 1e3, 3), "rtol": w.tol,
            "note": "best of %d; backward = adjoint BRAS-PCG + per-element contraction" % steps}


def mfma_section(prob, w, bras_us, iters=400, blocks=2048):
    """BF16 apply: matrix-core FLOPs of the full apply against the BF16 peak,
    and the LDS-resident microbenchmark of its element-local Gram products."""
    import torch
    from paper_2607_12138_amd import _lib as L
    nl, R = prob.n_loc, w.nrhs
    per_round = L.bras_bench_bf16_local_gemm(nl, 1, 0)          # one element, 32 columns, zero padding included
    issued = per_round * prob.E * ((R + 31) // 32)
    useful = 2.0 * nl * (nl + 1) * R * prob.E                   # the two triangular products
    out = torch.empty(blocks * 256, dtype=torch.float32, device="cuda")
    L.bras_bench_bf16_local_gemm(nl, 10, blocks, out)            # warm-up
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    flops = L.bras_bench_bf16_local_gemm(nl, iters, blocks, out)
    ev[1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1])
    mb = flops / (ms * 1e-3) / 1e12
    return {"full_apply": {"issued_tflops": round(issued / (bras_us * 1e-6) / 1e12, 2),
                           "useful_tflops": round(useful / (bras_us * 1e-6) / 1e12, 2),
                           "peak_tflops": BF16_PEAK_TFLOPS,
                           "frac_issued": round(issued / (bras_us * 1e-6) / 1e12 / BF16_PEAK_TFLOPS, 4)},
            "local_gemm_microbenchmark": {
                "label": "microbenchmark: element-local Gram products on LDS-resident tiles, no HBM traffic",
                "blocks": blocks, "rounds_per_block": iters, "ms": round(ms, 3), "issued_tflops": round(mb, 1),
                "frac_of_bf16_peak": round(mb / BF16_PEAK_TFLOPS, 4),
                "useful_fraction_of_issued": round(useful / issued, 4)}}


def setup_section(prob):
    """Time of bras_update (element coefficients -> per-element FP64
    Cholesky, triangular inverse and folded inverse or Gram factor, and
    diag(M)), against the FP64 peak: about n_loc^3 flops per element (n^3/3
    each for the factorisation, the triangular inverse and the product of the
    inverse factors)."""
    import torch
    from paper_2607_12138_amd import _lib as L
    reps = 3
    best = None
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        L.bras_update(prob.h, prob.elem_d)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        best = dt if best is None else min(best, dt)
    flop = float(prob.E) * prob.n_loc ** 3
    if prob.form == L.ELEM_SCALED_REF:
        flop = float(prob.n_loc) ** 3   # one shared reference inverse (the rest is per-element scaling)
    tf = flop / best / 1e12
    return {"update_ms": round(best * 1e3, 3), "gflop": round(flop / 1e9, 3), "tflops": round(tf, 4),
            "frac_fp64_peak": round(tf / FP64_PEAK_TFLOPS, 5)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=DEFAULT, choices=sorted(workloads.BY_NAME))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--apply-reps", type=int, default=50)
    ap.add_argument("--no-assembled", action="store_true", help="skip the assembled (CSR) BRAS comparison and the Schur-complement products")
    ap.add_argument("--stationary-steps", type=int, default=2,
                    help="timed fixed-point / Chebyshev solves of each kind (0: skip)")
    ap.add_argument("--mode", choices=["full", "apply", "mass", "copy", "solve"], default="full",
                    help="apply / mass: only back-to-back BRAS / mass applies (for counter runs); "
                         "copy: a device copy of known size (counter calibration); "
                         "solve: only BRAS-PCG solves (for kernel traces of the solve)")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py runs on exactly one GPU: the method has no multi-GPU path in this library "
              "(--gpus %d requested)" % a.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2607_12138_amd import _lib as L
    from paper_2607_12138_amd.problem import MassProblem

    if a.mode == "copy":
        nbytes = 1 << 30
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(a.apply_reps):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "copy", "bytes_read": nbytes, "bytes_written": nbytes, "reps": a.apply_reps}))
        return

    w = workloads.BY_NAME[a.workload]
    rho = workloads.density(w.n_cells, w.seed(2)) if w.density else None
    t0 = time.perf_counter()
    prob = MassProblem(w.family, w.dim, w.degree, w.N, jitter=w.jitter, seed=w.mesh_seed, rho=rho, prec=w.prec,
                       max_rhs=w.nrhs)
    variant = prob.autotune(w.nrhs) if a.mode == "full" else -1
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    print("setup done: n=%d E=%d n_loc=%d (%.1f s)" % (prob.n, prob.E, prob.n_loc, setup_s), file=sys.stderr,
          flush=True)
    b_host = workloads.rhs(prob.n, w.nrhs, w.seed(1))
    b = torch.from_numpy(b_host).cuda()
    if a.mode == "mass":
        y = prob.vec(w.nrhs)
        us = time_apply(lambda u, v: L.mass_apply(prob.h, u, v), b, y, a.apply_reps)
        prob.close()
        print(json.dumps({"mode": "mass", "workload": w.name, "reps": a.apply_reps, "us_per_apply": round(us, 3),
                          "source_digest": source_digest(w)}), flush=True)
        return
    if a.mode == "apply":
        y = prob.vec(w.nrhs)
        us = time_apply(lambda u, v: L.bras_apply(prob.h, u, v), b, y, a.apply_reps)
        prob.close()
        print(json.dumps({"mode": "apply", "workload": w.name, "reps": a.apply_reps, "us_per_apply": round(us, 3),
                          "bytes_per_apply": int(algorithmic_bytes(w, prob.n, prob.E, prob.n_loc, w.nrhs, w.prec)),
                          "source_digest": source_digest(w)}), flush=True)
        return
    if a.mode == "solve":
        for _ in range(a.warmup):
            prob.solve(b, "bras", rtol=w.tol)
        ms, st, its, rel, _ = time_solves(prob, b, "bras", w.tol, a.steps)
        prob.close()
        print(json.dumps({"mode": "solve", "workload": w.name, "steps": a.steps, "ms_per_solve": round(ms, 4),
                          "iterations": [int(v) for v in its], "source_digest": source_digest(w)}), flush=True)
        return
    for _ in range(a.warmup):
        prob.solve(b, "bras", rtol=w.tol)
        prob.solve(b, "jacobi", rtol=w.tol)
    print("warmup done", file=sys.stderr, flush=True)
    bras_ms, st_b, its_b, rel_b, xb = time_solves(prob, b, "bras", w.tol, a.steps)
    jac_ms, st_j, its_j, rel_j, xj = time_solves(prob, b, "jacobi", w.tol, a.steps)
    print("solves done: bras %.3f ms (%s its), jacobi %.3f ms (%s its)" % (bras_ms, its_b, jac_ms, its_j),
          file=sys.stderr, flush=True)
    stat = None
    if a.stationary_steps > 0:
        stat = stationary_section(prob, b, w, a.stationary_steps)
        print("stationary done: %s" % json.dumps(stat), file=sys.stderr, flush=True)
    x = prob.vec(w.nrhs)
    x.copy_(b)
    y = prob.vec(w.nrhs)
    bras_us = time_apply(lambda u, v: L.bras_apply(prob.h, u, v), x, y, a.apply_reps)
    mass_us = time_apply(lambda u, v: L.mass_apply(prob.h, u, v), x, y, a.apply_reps)
    cold_us = time_apply_cold(lambda u, v: L.bras_apply(prob.h, u, v), x, y, 20)
    copy_gbs = device_copy_gbs()
    nbytes = algorithmic_bytes(w, prob.n, prob.E, prob.n_loc, w.nrhs, w.prec)
    achieved = nbytes / (bras_us * 1e-6) / 1e9
    assembled = None
    schur = None
    if w.nrhs == 1 and w.prec != "bf16" and not a.no_assembled:
        assembled = assembled_section(prob, x, y, bras_us, a.apply_reps)
        print("assembled done: %s" % json.dumps(assembled), file=sys.stderr, flush=True)
        schur = schur_section(prob, w)
        print("schur done: %s" % json.dumps(schur), file=sys.stderr, flush=True)
    y_b0 = None
    rows = y_rows = None
    if not a.no_cpu_baseline:
        yb = prob.vec(w.nrhs)
        L.bras_apply(prob.h, b, yb)
        y_b0 = (yb if w.nrhs == 1 else yb[:, 0]).cpu().numpy()
        if w.prec == "bf16":
            rows = np.sort(np.random.default_rng(w.seed(4)).choice(prob.n, 256, replace=False))
            y_rows = yb[torch.from_numpy(rows).cuda()].cpu().numpy()
    grad = gradient_section(prob, w, b) if w.density else None
    if grad:
        print("gradient done: %s" % json.dumps(grad), file=sys.stderr, flush=True)
    setup_upd = setup_section(prob)
    mfma = mfma_section(prob, w, bras_us) if w.prec == "bf16" else None
    traffic = stored_traffic(w.name)
    out = {
        "metric": METRIC,
        "value": round(bras_ms, 4),
        "unit": "ms (BRAS-PCG time to solution)",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(bras_ms, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f64": "f64", "f32": "f32 apply / f64 CG", "bf16": "bf16 apply / f64 CG"}[w.prec],
        "data": "synthetic: seeded Kuhn mesh and U[-1,1] right-hand side",
        "config": {
            "workload": w.name, "family": {"P": "H1 Lagrange", "B": "H1 Bernstein", "N1curl": "N1curl", "RT": "RT",
                                           "N2curl": "N2curl", "BDM": "BDM"}[w.family],
            "degree": w.degree, "dim": w.dim, "mesh": "%d^%d Kuhn simplices, jitter %.1fh" % (w.N, w.dim, w.jitter),
            "n": prob.n, "E": prob.E, "n_loc": prob.n_loc, "nrhs": w.nrhs, "rtol": w.tol, "apply_precision": w.prec,
        },
        "jacobi_ms": round(jac_ms, 4),
        "speedup_vs_jacobi": round(jac_ms / bras_ms, 3),
        "iterations": {"bras": [int(v) for v in its_b], "jacobi": [int(v) for v in its_j]},
        "true_relres": {"bras": float(np.max(rel_b)), "jacobi": float(np.max(rel_j))},
        "bras_apply_us": round(bras_us, 3),
        "mass_apply_us": round(mass_us, 3),
        "bras_apply_gbs": round(achieved, 1),
        "bras_apply_cold_us": round(cold_us, 3),
        "bras_apply_cold_gbs": round(nbytes / (cold_us * 1e-6) / 1e9, 1),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": ("bras_apply (patch pass k_patch + shared-DOF pass k_patch_shared)"
                                if prob.info("patches") > 0 else "bras_apply (element pass + transpose-map reduce)"),
                     "bytes_per_launch": int(nbytes), "us_per_launch": round(bras_us, 3),
                     "copy_gbs": round(copy_gbs, 1), "frac_of_copy": round(achieved / copy_gbs, 4)},
        "source_digest": source_digest(w),
        "setup_s": round(setup_s, 3),
        "element_pass_variant": int(variant),
        "stationary": stat,
        "assembled_bras": assembled,
        "schur_bras": schur,
        "element_setup": setup_upd,
        "gradient": grad,
        "mfma": mfma,
        "patches": int(prob.info("patches")),
        "autotune": {"variant": int(variant), "patch_form": int(prob.info("patch_on")),
                     "note": "bras_autotune's pick among the element-pass variants and the patch form"},
    }
    if not a.no_cpu_baseline:
        print("cpu baseline ...", file=sys.stderr, flush=True)
        if w.prec == "bf16":
            extra, out["cpu_baseline"] = cpu_baseline_sampled(w, int(max(its_b)), rows, y_rows)
        else:
            extra, out["cpu_baseline"] = cpu_baseline(w, int(max(its_b)), y_gpu=y_b0)
        prec = {"apply_precision": w.prec}
        prec.update(extra)
        if "oracle_iterations" in extra:
            prec["iterations_gpu_minus_oracle"] = int(its_b[0]) - extra["oracle_iterations"]
        out["precision_vs_fp64_oracle"] = prec
    prob.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
