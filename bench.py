"""Benchmark: TE solves/s to a true FP64 relative residual of 1e-8 on one MI355X.

Headline workload: the 256 x 256 size class of the batched random-field workload --
four objects (seeds 1004..1007: Re eps = 1 + 9U, Im eps = 0.5 U2, correlation length
lambda/2, masked to a random ellipse; h = lambda/48, so 5.33 wavelengths across) lit
by 64 equispaced TE plane waves each: 256 solves.  A step solves all 256 in one
die_te_solve_batch call over four single-object contexts (a host thread and a stream each):
block GMRES(30) with one block Krylov space per object (complex64 products and basis;
the two block Gram-Schmidt passes of each step as binary16 GEMMs on planar copies of the
basis with FP32 accumulation, CholQR of each new block (its Gram on the matrix cores, the
factor on the device, a second pass only for ill-conditioned blocks), FP64 block least squares; --block-gemm 32 keeps the Gram-Schmidt GEMMs in complex64 with one pass,
--block-precision 64 runs everything in complex128), every cycle restarted from the FP64
true residual, tol 1e-8 on that residual, zero initial guess.  --solver rhs times the per-rhs batched solver instead
(one-reduction Arnoldi, complex binary16 basis; --basis 32 / --orth 0 select the
complex64 basis and the two-pass CGS2); it is also reported beside the block run.  Inputs are resident in HBM before the timed region; the
per-object setup (symbol) is done once, outside it.

The configured deflation (k = 16 largest-magnitude eigenvalues per object) is not applied in
the headline: with the block solver it converges every solve but takes more block steps (and its
eigensolver setup), and with one-vector GMRES(30) on A P^-1 many angles stagnate near 3e-2 (an
independent scipy GMRES(30) with ARPACK eigenvectors stagnates at the same value).  So the
headline and the plain baseline both solve the undeflated system A, and the same batch with
k = 16 is reported beside them (configured_deflation_k16).

Reported next to it: the plain solver (FP64 products and basis, one right-hand side per
call, the same GMRES(30) and orthogonalisation, a sample of 16 of the 256 solves), the product throughput at the batched shape and at
the 1024^2 class (64 fields), the hard-cylinder variants (regularizer, deflation,
mixed precision), the learned warm start (the stored configured network's guesses, its
inference inside the timed region, then the same batched solve), the uneven configuration (16
objects in four size classes 128^2 .. 1024^2, 64 angles each, 1024 solves in one call per
restart-cycle chunk, within a wall-clock budget) and the FP64 oracle on the host.

One JSON line on stdout; progress on stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {16: 2500.0, 32: 157.3, 64: 78.6}  # dense matrix-core peaks: fp16, fp32, fp64
N_ANGLES = 64
OBJ_SEEDS = (1004, 1005, 1006, 1007)
RESTART = 30
TOL = 1e-8
MAX_ITERS = 20000


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def product_model_bytes(nx, ny, px, py, nrhs, elem_bytes, nobj=1):
    """3-pass model bytes of one operator product on nrhs fields: pass 1 reads u and chi
    and writes the row transforms of the ny rows; pass 2 reads and writes them and reads
    the 3-plane symbol; pass 3 reads them and u and writes y."""
    N = nx * ny
    return (2 * nrhs * N + nobj * N + 8 * nrhs * ny * px + 3 * px * py + 4 * nrhs * N) * elem_bytes


def source_hash(*names):
    h = hashlib.sha256()
    for nm in names:
        with open(os.path.join(ROOT, "paper_1104_4263_amd", "csrc", nm), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic(kernel_tag, src_hash, algorithmic_bytes):
    """HBM bytes per launch from a committed rocprofv3 --pmc summary: its measured ratio of
    HBM bytes (FETCH_SIZE + WRITE_SIZE, calibrated on a copy kernel) to algorithmic bytes,
    applied to this run's algorithmic bytes per launch.  None unless the summary was taken
    on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"{kernel_tag}_traffic.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith(" "):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256") != src_hash:
        return None
    try:
        return float(vals["hbm_over_algorithmic"]) * algorithmic_bytes
    except (KeyError, ValueError):
        return None


def cpu_info():
    """(BLAS threads, CPU model) of the host."""
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count() or 1
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return int(threads), model


def cpu_baseline(g, eps, n_angles):
    """The FP64 oracle on the host cores, as it stands: direct-sum products (O(N^2)) at 64^2
    and on the headline's 256^2 object, and the oracle's solver (dense assembly, LU factor,
    per-angle triangular solves) at 64^2 and 32^2.  The oracle cannot solve the 256^2 headline
    (its dense matrix would take 275 GB), so `value` is the 64^2 dense solve extrapolated to
    256^2 (assembly O(N^2), factorisation O(N^3), each angle's solve O(N^2)) with the
    factorisation shared by the object's n_angles angles, labelled as an extrapolation."""
    import numpy as np
    import scipy.linalg as sla
    from oracle import operator as op
    from synth import workload, plane_wave, centred_grid, cylinder
    threads, model = cpu_info()
    rng = np.random.default_rng(0)
    out = {}
    # (1) direct-sum products
    w = workload("cyl_small")
    g64, e64 = w["grids"][0], w["eps"][0]
    mv = {}
    for name, gg, ee in (("64x64 (small cylinder)", g64, e64), (f"{g.nx}x{g.ny} (headline object 0)", g, eps)):
        x = rng.standard_normal((2, gg.ny, gg.nx)) + 1j * rng.standard_normal((2, gg.ny, gg.nx))
        chi = op.electric_contrast(ee)
        reps = 0
        t0 = time.perf_counter()
        while True:
            op.apply_operator(gg, chi, x)
            reps += 1
            if time.perf_counter() - t0 > 1.0 or gg.nx > 64:
                break
        t = (time.perf_counter() - t0) / reps
        mv[name] = {"s": round(t, 4), "matvecs_per_s": round(1.0 / t, 4)}
        log(f"oracle direct-sum product {name}: {t:.3f} s")
    out["oracle_matvecs"] = mv
    # (2) dense solves: assembly, LU factor, per-angle solve
    lu = {}
    t64 = None
    for n, gg, ee in ((64, g64, e64), (32, None, None)):
        if gg is None:
            gg = centred_grid(n, 0.6)
            ee = cylinder(gg, 0.25, 4.0 + 0j)
        t0 = time.perf_counter()
        A = op.dense_operator(gg, op.electric_contrast(ee))
        t1 = time.perf_counter()
        f = sla.lu_factor(A, overwrite_a=True, check_finite=False)
        t2 = time.perf_counter()
        bs = np.stack([plane_wave(gg, 2.0 * math.pi * j / 8).ravel() for j in range(8)], axis=1)
        sla.lu_solve(f, bs, check_finite=False)
        t3 = time.perf_counter()
        per_angle = (t3 - t2) / 8
        lu[f"{n}x{n}"] = {"assemble_s": round(t1 - t0, 3), "factor_s": round(t2 - t1, 3),
                          "solve_per_angle_s": round(per_angle, 5),
                          "solves_per_s_one_angle": round(1.0 / (t3 - t0 - 7 * per_angle), 4),
                          f"solves_per_s_{n_angles}_angles": round(n_angles / (t2 - t0 + n_angles * per_angle), 4)}
        if n == 64:
            t64 = (t1 - t0, t2 - t1, per_angle)
        log(f"oracle dense solve {n}x{n}: {lu[f'{n}x{n}']}")
        del A, f
    out["oracle_dense_solves"] = lu
    # (3) the 256^2 headline by extrapolation from 64^2
    q = (g.nx * g.ny) / (64.0 * 64.0)
    t_obj = t64[0] * q * q + t64[1] * q ** 3 + n_angles * t64[2] * q * q
    value = n_angles / t_obj
    total = sum(v["s"] for v in mv.values()) + sum(v["assemble_s"] + v["factor_s"] for v in lu.values())
    out.update({"value": value, "unit": "solves/s", "cores": threads, "kind": "oracle",
                "cpu_model": model, "blas_threads": threads,
                "sample": (f"oracle dense LU solve at 64x64 (assembly {t64[0]:.1f} s, factor {t64[1]:.1f} s, "
                           f"{t64[2] * 1e3:.1f} ms per angle) extrapolated to the {g.nx}x{g.ny} headline "
                           f"(assembly x{q * q:.0f}, factor x{q ** 3:.0f}, per-angle solve x{q * q:.0f}; "
                           f"{n_angles} angles per factorisation): an extrapolation, the 256^2 dense matrix "
                           f"needs 275 GB; measured oracle figures beside it ({total:.1f} s of CPU work)"),
                "extrapolated": True})
    return out


def learned_leg(solve, ctxs, Bs, steps, nsolve, value_zero, iters_zero, plain_value):
    """The configured warm-start network (stored parameters, trained on 20 032 block-solver solves
    of objects the headline never uses) guessing the headline batch: network inference and the
    same batched solve from its guesses, timed together over `steps` batches after one warm-up."""
    import numpy as np
    import torch
    from paper_1104_4263_amd import warm_start
    try:
        net = warm_start.load_network(max_batch=64)
    except (FileNotFoundError, ValueError) as e:
        return {"skipped": str(e)}
    with open(warm_start.RECORD_PATH) as f:
        rec = json.load(f)

    def guess_and_solve():
        x0s = [net.warm_start(c, b) for c, b in zip(ctxs, Bs)]
        return x0s, solve(x0s)

    guess_and_solve()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        x0s, (us, rc, info) = guess_and_solve()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    # inference alone
    t1 = time.perf_counter()
    for c, b in zip(ctxs, Bs):
        net.warm_start(c, b)
    torch.cuda.synchronize()
    inf_s = time.perf_counter() - t1
    ok = rc == 0 and all(x["rel_res_true"] <= TOL for x in info)
    it = np.array([x["iters"] for x in info])
    e_net, e_inc = [], []
    for x0, u, b in zip(x0s, us, Bs):
        for r in range(b.shape[0]):
            nu = torch.linalg.vector_norm(u[r]).item()
            e_net.append(torch.linalg.vector_norm(x0[r] - u[r]).item() / nu)
            e_inc.append(torch.linalg.vector_norm(b[r] - u[r]).item() / nu)
    v = nsolve / dt if ok else 0.0
    net.close()
    return {"value": round(v, 3), "unit": "solves/s", "ms_per_step": round(1000.0 * dt, 2),
            "method": "the headline's batched solver started from the network's guesses (network inference inside "
                      "the timed region)",
            "network": rec["network"], "training": {**rec["data"], **{k: rec["training"][k] for k in
                                                                      ("epochs", "steps", "train_s", "TFLOPs")}},
            "inference_s": round(inf_s, 4), "iters_mean": round(float(it.mean()), 1), "iters_max": int(it.max()),
            "iters_mean_zero_guess": round(float(iters_zero.mean()), 1),
            "iters_max_zero_guess": int(iters_zero.max()),
            "guess_rel_err_median": round(float(np.median(e_net)), 4),
            "incident_rel_err_median": round(float(np.median(e_inc)), 4),
            "rel_res_true_max": max(x["rel_res_true"] for x in info),
            "vs_zero_guess": round(v / value_zero, 3) if value_zero > 0 else None,
            "vs_plain": round(v / plain_value, 2) if plain_value else None}


SIZE_CLASSES = (128, 256, 512, 1024)  # object o of the batched workload has size class o // 4, seed 1000 + o


def uneven_run(sizes, args, deflate_k=0, budget_s=None):
    """Several size classes of the batched workload (4 objects x 64 angles each) solved in one
    die_te_solve_batch call: one context per object with the block solver and --contexts
    per-object (classes up to 256^2), else one context per grid size.  deflate_k: the deflation
    size of every object (eigensolver setup timed apart); budget_s: stop after the chunk that
    passes this many seconds and report the state reached."""
    import numpy as np
    import torch
    from synth import plane_wave, random_field_object
    from paper_1104_4263_amd import Solver
    solvers, Bs, cls = [], [], []
    per_object = args.solver == "block" and args.contexts == "per-object"
    t_setup = time.perf_counter()
    for n in sizes:
        c = SIZE_CLASSES.index(n)
        objs = [random_field_object(n, seed=1000 + 4 * c + i) for i in range(4)]
        gn = objs[0][0]
        b1 = torch.from_numpy(np.stack([plane_wave(gn, 2.0 * math.pi * j / N_ANGLES) for j in range(N_ANGLES)])).cuda()
        dk = dict(deflate_k=deflate_k, seed=1) if deflate_k else {}
        if per_object and n <= 256:  # larger classes: one context per class (block buffers of one object at a time)
            for _, e in objs:
                solvers.append(Solver.from_grid(gn, e, **dk))
                Bs.append(b1)
                cls.append(n)
        else:
            solvers.append(Solver.from_grid(gn, np.stack([e for _, e in objs]), **dk))
            Bs.append(torch.cat([b1] * 4))
            cls.append(n)
        log(f"uneven: class {n} set up ({time.perf_counter() - t_setup:.1f} s)")
    if args.solver == "block":
        kw = dict(restart=RESTART, tol=TOL, mixed=1 if args.block_precision == 32 else 0,
                  block=2 if args.block_gemm == 16 else 1, orth=args.block_orth)
    else:
        kw = dict(restart=RESTART, tol=TOL, mixed=2 if args.basis == 16 else 1, orth=args.orth)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t_setup
    Solver.solve_batch(solvers, Bs, max_iters=RESTART, **kw)  # allocates every context's buffers
    torch.cuda.synchronize()
    # solved in chunks of two restart cycles, each starting from the previous chunk's fields (the
    # restart the next cycle would make anyway), so that every chunk reports its progress
    X = [torch.zeros_like(b) for b in Bs]
    iters = [np.zeros(b.shape[0], dtype=np.int64) for b in Bs]
    t0 = time.perf_counter()
    rc, chunk = 1, 2 * RESTART
    stopped = False
    while rc != 0 and int(max(i.max() for i in iters)) < MAX_ITERS:
        if budget_s is not None and time.perf_counter() - t0 > budget_s:
            stopped = True
            break
        res, rc = Solver.solve_batch(solvers, Bs, x0s=X, inplace=True, max_iters=chunk, **kw)
        X = [u for u, _ in res]
        for c, (_, inf) in enumerate(res):
            iters[c] += np.array([x["iters"] for x in inf])
        worst = {n: max(max(x["rel_res_true"] for x in inf) for (_, inf), cn in zip(res, cls) if cn == n)
                 for n in sizes}
        log(f"uneven: {time.perf_counter() - t0:.1f} s, worst rel-res per class "
            f"{', '.join(f'{n}: {w:.1e}' for n, w in worst.items())}")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    nsol = sum(b.shape[0] for b in Bs)
    ok = rc == 0 and all(x["rel_res_true"] <= TOL for _, inf in res for x in inf)
    per = {}
    for n in sizes:
        it = np.concatenate([i for i, cn in zip(iters, cls) if cn == n])
        rr = [x["rel_res_true"] for (_, inf), cn in zip(res, cls) if cn == n for x in inf]
        per[f"{n}x{n}"] = {"iters_mean": round(float(np.mean(it)), 1), "iters_max": int(it.max()),
                           "converged": int(sum(r <= TOL for r in rr)), "of": len(rr),
                           "worst_rel_res": max(rr)}
    out = {"workload": f"size classes {sizes} of the batched random-field workload, 4 objects x {N_ANGLES} "
                       f"angles each, die_te_solve_batch calls of two restart cycles each over "
                       f"{len(solvers)} contexts", "solver": args.solver, "deflate_k": deflate_k,
           "setup_s": round(setup_s, 1), "solves": nsol,
           "s": round(dt, 3), "finished": ok, "stopped_at_budget_s": budget_s if stopped else None,
           "solves_per_s": round(nsol / dt, 3) if ok else 0.0, "classes": per}
    log(f"uneven: {out}")
    for sv in solvers:
        sv.close()
    return out


# The paper's Table 2 (TE, tol 1e-8 on the solved system, fair memory: restart + r = 40): per
# object (eps of the square) and system, the deflation size r, the restart and the iterations.
# The paper's Table 1 (TM, fair memory): per square, the deflation size r, the restart and the iterations.
PAPER_TABLE1 = {
    "16": {"A": (0, 40, 7311), "A P^-1": (28, 12, 4230)},
    "-16+1.5i": {"A": (0, 40, 27), "A P^-1": (28, 12, 14)},
    "16 with a 2.5+20i core": {"A": (0, 40, 1000), "A P^-1": (28, 12, 749)},
}
PAPER_TABLE2 = {
    "16": {"A": (0, 40, 15258), "A P^-1": (6, 34, 14002), "A_R A": (0, 40, 4030), "A_R A P^-1": (14, 26, 3626)},
    "-16+1.5i": {"A": (0, 40, 1708), "A P^-1": (7, 33, 1659), "A_R A": (0, 40, 1021), "A_R A P^-1": (30, 10, 534)},
    "16 with a 2.5+20i core": {"A": (0, 40, 11823), "A P^-1": (3, 37, 13156), "A_R A": (0, 40, 3032),
                               "A_R A P^-1": (14, 26, 2911)},
}


def method_variants(cap_reg=24000, long_k=(20, 40)):
    """The paper's four systems A, A P^-1, A_R A and A_R A P^-1 (per-rhs GMRES, FP64 and mixed
    precision) on three workloads: the hard cylinder (256^2, eps = -2.5+0.2i, psi = 30 deg), its
    half-size analog (128^2 over 2.2 lambda, radius 1 lambda, same eps and cell size) and the three
    squares of the paper's Table 2 at 61^2 nodes with the table's r and restart.  Every solve is
    accepted on the FP64 true residual; the paper's iteration counts are context only (its 3N system
    and its regularized residual)."""
    import numpy as np
    import torch
    from synth import workload, plane_wave, plane_wave_te3, plane_wave_tm, centred_grid, cylinder
    from paper_1104_4263_amd import Solver

    def run(g, e, b, reg, k, restart, cap, mixed, seed=1, memory=None, method="gmres", **kw):
        """k = -1: automatic deflation size; memory: restart = memory - r (fair memory); method:
        the Krylov solver; kw: the system (polarization, magnetic)."""
        t0 = time.perf_counter()
        sv = Solver.from_grid(g, e, regularize=reg, deflate_k=k, seed=seed, **kw)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if k == -1:
            ritz, _, _ = sv.deflation_info()
            k = int((ritz.abs() > 0).sum())
            if memory is not None:
                restart = max(memory - k, 5)
        _, rc, inf = sv.solve(b, restart=restart, max_iters=cap, tol=TOL, mixed=mixed, method=method)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        sv.close()
        i = inf[0]
        return {"converged": rc == 0, "iters": i["iters"], "products_A": i["products_A"],
                "products_AR": i["products_AR"], "rel_res_true": i["rel_res_true"], "restart": restart, "k": k,
                "setup_s": round(t1 - t0, 3), "solve_s": round(t2 - t1, 4)}

    out = {}
    systems = (("A", False, False), ("A P^-1", False, True), ("A_R A", True, False), ("A_R A P^-1", True, True))
    # hard cylinder and its half-size analog: GMRES(30), k = 20
    w = workload("cyl_hard")
    cases = {"cylinder 256^2 (r = 2 lambda, eps = -2.5+0.2i, psi = 30 deg)": (w["grids"][0], w["eps"][0])}
    gh = centred_grid(128, 2.2)
    cases["cylinder 128^2 half-size analog (r = 1 lambda, same eps and h)"] = (gh, cylinder(gh, 1.0, -2.5 + 0.2j))
    for cname, (gc, ec) in cases.items():
        bc = torch.from_numpy(plane_wave(gc, math.pi / 6.0)).cuda()
        res = {}
        for name, reg, defl in systems:
            for mixed in (False, True):
                cap = cap_reg if reg else MAX_ITERS
                key = name + (" mixed" if mixed else "")
                res[key] = run(gc, ec, bc, reg, 20 if defl else 0, 30, cap, mixed)
                log(f"{cname} {key}: {res[key]}")
        out[cname] = res
    # the hard cylinder's regularized systems with the larger deflation sizes
    gc, ec = w["grids"][0], w["eps"][0]
    bc = torch.from_numpy(plane_wave(gc, math.pi / 6.0)).cuda()
    extra = {}
    for k in long_k:
        if k == 20:
            continue
        key = f"A_R A P^-1, k = {k}"
        extra[key] = run(gc, ec, bc, True, k, 30, cap_reg, False)
        log(f"cylinder 256^2 {key}: {extra[key]}")
    out["cylinder 256^2 (r = 2 lambda, eps = -2.5+0.2i, psi = 30 deg)"].update(extra)
    # the paper's squares (side lambda, 61^2 nodes), psi = 0, with Table 2's r and restart
    ws = workload("paper_squares")
    gs = ws["grids"][0]
    bs = torch.from_numpy(plane_wave(gs, 0.0)).cuda()
    for label, es in zip(PAPER_TABLE2, ws["eps"]):
        res = {}
        for name, reg, defl in systems:
            r, restart, paper_it = PAPER_TABLE2[label][name]
            for mixed in (False, True):
                key = name + (" mixed" if mixed else "")
                res[key] = run(gs, es, bs, reg, r, restart, MAX_ITERS if not reg else cap_reg, mixed)
                res[key]["paper_iters"] = paper_it
                log(f"square eps = {label} {key}: {res[key]}")
        # Section 5's automatic deflation size (radius rule) with the fair-memory restart 40 - r
        res["A_R A P^-1, automatic r"] = run(gs, es, bs, True, -1, 0, cap_reg, False, memory=40)
        res["A_R A P^-1, automatic r"]["deflation_radius"] = round(
            __import__("paper_1104_4263_amd").die_te_deflation_radius(es, True), 4)
        log(f"square eps = {label} automatic r: {res['A_R A P^-1, automatic r']}")
        out[f"Table 2 square, eps = {label} (61^2 nodes)"] = res
    # Table 2 on the paper's own 3N system (E1, E2, H3; no magnetic contrast): counts comparable to the table
    b3 = torch.from_numpy(plane_wave_te3(gs, 0.0)).cuda()
    for label, es in zip(PAPER_TABLE2, ws["eps"]):
        res = {}
        for name, reg, defl in systems:
            r, restart, paper_it = PAPER_TABLE2[label][name]
            res[name] = run(gs, es, b3, reg, r, restart, cap_reg if reg else MAX_ITERS, False, magnetic=True)
            res[name]["paper_iters"] = paper_it
            log(f"3N square eps = {label} {name}: {res[name]}")
        out[f"Table 2 square, eps = {label}, the 3N (E1, E2, H3) system"] = res
    # Table 1: the TM squares, unpreconditioned against deflated (r = 28, restart 12), and the
    # automatic size (every eigenvalue outside the unit circle) with the fair-memory restart
    btm = torch.from_numpy(plane_wave_tm(gs, 0.0)).cuda()
    for label, es in zip(PAPER_TABLE1, ws["eps"]):
        res = {}
        for name, defl in (("A", False), ("A P^-1", True)):
            r, restart, paper_it = PAPER_TABLE1[label][name]
            res[name] = run(gs, es, btm, False, r, restart, MAX_ITERS, False, polarization="tm")
            res[name]["paper_iters"] = paper_it
            log(f"TM square eps = {label} {name}: {res[name]}")
        res["A P^-1, automatic r"] = run(gs, es, btm, False, -1, 0, MAX_ITERS, False, memory=40, polarization="tm")
        log(f"TM square eps = {label} automatic r: {res['A P^-1, automatic r']}")
        out[f"Table 1 square (TM), eps = {label} (61^2 nodes)"] = res
    # the Conclusions' alternatives to restarted GMRES on the regularized, deflated system (Table 2's
    # r; GMRES and GCR with the table's restart, Bi-CGSTAB, IDR(4)); iters count applications of M
    for label, es in zip(PAPER_TABLE2, ws["eps"]):
        r, restart, _ = PAPER_TABLE2[label]["A_R A P^-1"]
        res = {}
        for meth, rs in (("gmres", restart), ("bicgstab", restart), ("gcr", restart), ("idrs", 4)):
            res[meth] = run(gs, es, bs, True, r, rs, cap_reg, False, method=meth)
            log(f"square eps = {label} A_R A P^-1 {meth}: {res[meth]}")
        out[f"Krylov solvers on A_R A P^-1, Table 2 square eps = {label}"] = res
    out["spectra (Figs. 2 and 3), Table 2 squares at 21^2 nodes"] = spectra_summary()
    return out


def spectra_summary(nodes=21):
    """Eigenvalues of A (TE and TM) and of A_R A (TE) for the three squares of Table 2 on a coarse
    grid, summarised as the paper reads its Figs. 2 and 3: the share of eigenvalues on the far
    three quarters of the dense segments [1, eps] (for A_R A their images under eq.
    EigenvaluesArA; a TM spectrum only accumulates at 1), the largest magnitude and the number
    beyond Section 5's deflation radius."""
    import numpy as np
    from synth import workload
    from paper_1104_4263_amd import Solver, die_te_deflation_radius
    ws = workload("paper_squares", nodes=nodes)
    g = ws["grids"][0]
    out = {}

    def near(lam, segs, tol):
        """share of lam within tol of the polyline segs, beyond its first quarter (by length)"""
        lens = np.array([abs(b - a) for a, b in segs])
        start = np.concatenate([[0.0], np.cumsum(lens)[:-1]])
        total = max(float(lens.sum()), 1e-300)
        hit = np.zeros(lam.shape, dtype=bool)
        for (a, b), s0, ln in zip(segs, start, lens):
            t = np.clip(((lam - a) * np.conj(b - a)).real / max(ln ** 2, 1e-300), 0.0, 1.0)
            hit |= (np.abs(lam - (a + t * (b - a))) <= tol) & ((s0 + t * ln) >= 0.25 * total)
        return float(np.mean(hit))

    for label, es in zip(PAPER_TABLE2, ws["eps"]):
        vals = np.unique(np.round(es[es != 1.0], 12))
        res = {}
        for pol, reg, which in (("te", False, "A"), ("te", True, "ARA"), ("tm", False, "A")):
            t0 = time.perf_counter()
            sv = Solver.from_grid(g, es, regularize=reg, polarization=pol)
            lam = sv.spectrum(which)
            sv.close()
            segs = []
            for e in vals:
                if which == "ARA":  # the image of [1, e] under lam -> (1 + (1 - lam) / e) lam, as a polyline
                    t = np.linspace(0.0, 1.0, 65)
                    pts = 1.0 + t * (e - 1.0)
                    pts = (1.0 + (1.0 - pts) / e) * pts
                    segs += list(zip(pts[:-1], pts[1:]))
                else:
                    segs.append((1.0 + 0j, complex(e)))
            scale = max(1.0, max(abs(e - 1.0) for e in vals))
            radius = die_te_deflation_radius(es, reg) if pol == "te" else 1.0
            key = f"{'TE' if pol == 'te' else 'TM'} {which}"
            res[key] = {"unknowns": int(lam.size), "max_abs": round(float(np.abs(lam).max()), 4),
                        "share_on_segments": round(near(lam, segs, 0.02 * scale), 4),
                        "deflation_radius": round(float(radius), 4),
                        "beyond_radius": int(np.sum(np.abs(lam) > radius * (1 + 1e-9))),
                        "seconds": round(time.perf_counter() - t0, 2)}
            log(f"spectrum square eps = {label} {key}: {res[key]}")
        out[f"eps = {label}"] = res
    return out


PRODUCT_SRC = ("kernels_fft.hip", "fft.hpp", "ops.hpp", "common.hpp")  # the product kernels and their headers


def product_roofline(n=1024, nrhs=64, reps=10):
    """Roofline of the operator product (the three FFT pass kernels of one application of A)
    on nrhs complex64 fields of an n x n grid (px = py = 2n), the size whose working set is far
    beyond the 256 MB last-level cache: algorithmic bytes (22 R + 1) N s + 3 P s per launch of
    the three passes, divided by their average duration from HIP events recorded on the stream
    the library launches them on."""
    import torch
    from synth import centred_grid, cylinder
    from paper_1104_4263_amd import Solver
    gl = centred_grid(n, n / 48.0)
    sl = Solver.from_grid(gl, cylinder(gl, n / 48.0 / 3.0, 4.0))
    x = torch.randn(nrhs, 2, n, n, dtype=torch.complex64, device="cuda")
    ms = time_matvec(sl, x, reps)
    variants = sl.fft_plan(nrhs, torch.complex64)
    sl.close()
    del x
    mb = product_model_bytes(n, n, 2 * n, 2 * n, nrhs, 8)
    src = source_hash(*PRODUCT_SRC)
    traffic = read_traffic(f"fft_product_c64_{n}x{nrhs}", src, mb)
    gbs = mb / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None if traffic is None else int(traffic),
            "kernel": "operator product: die::k_rows_fwd + die::k_cols_symbol + die::k_rows_inv_sub",
            "workload": f"{n}x{n} cells (px = py = {2 * n}), {nrhs} complex64 fields, one object",
            "avg_launch_us": round(1000.0 * ms, 2), "algorithmic_bytes_per_launch": int(mb),
            "bytes_model": "(22 R + 1) N s + 3 P s (pass 1: 2RN + N read, 4RN written; pass 2: 4RN + 3P read, "
                           "4RN written; pass 3: 6RN read, 2RN written)",
            "matvecs_per_s": round(nrhs / ms * 1e3, 1), "fft_variants": variants, "kernel_source_sha256": src,
            "timing": f"HIP events on the launch stream around {reps} products after 2 warm-up products"}


def time_matvec(s, x, reps):
    """Average ms of one product call, timed with events on the stream the library launches on."""
    import torch
    for _ in range(2):
        s.matvec(x)
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        s.matvec(x)
    e1.record(st)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--solver", default="block", choices=("block", "rhs"),
                    help="block: block GMRES(30), one block Krylov space per object (default); rhs: per-rhs GMRES(30)")
    ap.add_argument("--block-precision", type=int, default=32, choices=(32, 64),
                    help="bits per real part of the block basis, GEMMs and products (32 with FP64 refinement, or 64)")
    ap.add_argument("--block-gemm", type=int, default=16, choices=(16, 32),
                    help="block solver: 16 = block Gram-Schmidt GEMMs on binary16 planar copies of the basis "
                         "(FP32 accumulation; needs --block-precision 32), 32 = complex GEMMs in the basis precision")
    ap.add_argument("--block-orth", type=int, default=None, choices=(0, 1),
                    help="block solver: 0 = two block Gram-Schmidt passes (default with --block-gemm 16), "
                         "1 = one pass (default with --block-gemm 32); CholQR2 of each new block either way")
    ap.add_argument("--contexts", default="per-object", choices=("per-object", "one"),
                    help="block solver: per-object = one context per object, all in one die_te_solve_batch call "
                         "(default); one = the single four-object context, objects one after another")
    ap.add_argument("--orth", type=int, default=1, choices=(0, 1),
                    help="Arnoldi orthogonalisation: 1 = one-reduction CGS2 (default), 0 = two-pass CGS2")
    ap.add_argument("--basis", type=int, default=16, choices=(16, 32),
                    help="bits per real part of the stored Krylov basis in the batched run (16 needs --orth 1)")
    ap.add_argument("--uneven-deflate", type=int, default=0, metavar="K",
                    help="--uneven: deflate the K largest-magnitude eigenvalues of every object")
    ap.add_argument("--uneven-budget", type=float, default=360.0, metavar="SECONDS",
                    help="--uneven: stop after the chunk that passes this many seconds of solving (0: no limit)")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned warm-start leg (the stored network's guesses + the batched solve)")
    ap.add_argument("--no-configured-deflation", action="store_true",
                    help="skip the headline batch with the configured k = 16 deflation per object")
    ap.add_argument("--product-only", action="store_true",
                    help="only time the operator product at 1024^2 x 64 fields (for profiling)")
    ap.add_argument("--variants-only", action="store_true",
                    help="only run the paper's four systems on the cylinders and Table 2's squares")
    ap.add_argument("--uneven", type=str, default="128,256,512,1024", metavar="SIZES",
                    help="size classes of the uneven batched configuration solved in one call ('' skips it)")
    args = ap.parse_args()
    if args.block_precision != 32:
        args.block_gemm = 32  # binary16 GEMMs only over a complex64 basis
    if args.block_orth is None:
        args.block_orth = 0 if args.block_gemm == 16 else 1
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the solver has no path across GPUs",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from synth import workload, plane_wave, centred_grid, cylinder, random_field_object
    from paper_1104_4263_amd import Solver
    from paper_1104_4263_amd._lib import DIE_PROF_PRODUCT, DIE_PROF_DOTS, DIE_PROF_AXPY, DIE_PROF_GEMM

    torch.cuda.set_device(0)
    if args.product_only:
        # the product kernels alone (for kernel traces and counters), then a 1 GiB copy whose
        # counters calibrate FETCH_SIZE and WRITE_SIZE
        r = product_roofline()
        x = torch.ones(2 ** 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        log("copy of 1073741824 bytes done")
        print(json.dumps({"roofline": r}), flush=True)
        return
    if args.variants_only:
        print(json.dumps({"method_variants": method_variants()}), flush=True)
        return
    objs = [random_field_object(256, seed=sd) for sd in OBJ_SEEDS]
    g = objs[0][0]
    eps = np.stack([e for _, e in objs])
    nobj = len(objs)
    psis = [2.0 * math.pi * j / N_ANGLES for j in range(N_ANGLES)]
    b1 = np.stack([plane_wave(g, p) for p in psis])
    B = torch.from_numpy(np.concatenate([b1] * nobj)).cuda()  # [object][angle] order
    nsolve = nobj * N_ANGLES

    block = args.solver == "block"
    t0 = time.perf_counter()
    s = Solver.from_grid(g, eps)  # one context holding the four objects (per-rhs solver, plain sample)
    # block solver: one context per object, all solved in one die_te_solve_batch call (a host
    # thread and a stream per context, so one object's host-side Cholesky factorisations and
    # one-workgroup least squares overlap the other objects' GEMMs and products)
    concurrent = block and args.contexts == "per-object"
    per_obj = [Solver.from_grid(g, eps[o]) for o in range(nobj)] if concurrent else []
    B_obj = [B[o * N_ANGLES:(o + 1) * N_ANGLES] for o in range(nobj)]
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    log(f"setup of {nobj} objects on {g.nx}x{g.ny}: {setup_s:.3f} s")
    timed_ctx = per_obj if concurrent else [s]

    def batch_solve(use_block=block, x0s=None):
        """The headline batch (x0s: one initial guess per timed context, else zero); returns the
        solutions per timed context (None for the per-object contexts unless guesses are given),
        the code and the records."""
        if use_block and not concurrent:
            u, rc, inf = s.solve(B, x0=None if x0s is None else x0s[0], restart=RESTART, max_iters=MAX_ITERS,
                                 tol=TOL, mixed=1 if args.block_precision == 32 else 0,
                                 block=2 if args.block_gemm == 16 else 1, orth=args.block_orth)
            return [u], rc, inf
        if use_block:
            res, rc = Solver.solve_batch(per_obj, B_obj, x0s=x0s, restart=RESTART, max_iters=MAX_ITERS, tol=TOL,
                                         mixed=1 if args.block_precision == 32 else 0,
                                         block=2 if args.block_gemm == 16 else 1, orth=args.block_orth)
            return ([u for u, _ in res] if x0s is not None else None), rc, [x for _, inf in res for x in inf]
        u, rc, inf = s.solve(B, x0=None if x0s is None else x0s[0], restart=RESTART, max_iters=MAX_ITERS, tol=TOL,
                             mixed=2 if args.basis == 16 else 1, orth=args.orth)
        return [u], rc, inf

    for i in range(args.warmup):
        _, rc, info = batch_solve()
        log(f"warmup {i}: rc {rc}, max iters {max(x['iters'] for x in info)}")
    torch.cuda.synchronize()
    for sv in timed_ctx:
        sv.profile(3)  # events around one launch in three of each kind (coprime with the per-iteration pattern)
    infos = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        _, rc, info = batch_solve()
        infos.append(info)
        log(f"step {i}: rc {rc}")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    for sv in timed_ctx:
        sv.profile(0)
    ms_per_step = 1000.0 * dt / args.steps
    last = infos[-1]
    converged = all(x["status"] == 0 and x["rel_res_true"] <= TOL for inf in infos for x in inf)
    value = nsolve * args.steps / dt if converged else 0.0
    iters = np.array([x["iters"] for x in last]).reshape(nobj, N_ANGLES)
    prods = np.array([x["products_A"] for x in last])
    log(f"timed {args.steps} batches of {nsolve} solves in {dt:.3f} s -> {value:.2f} solves/s; "
        f"iters per object mean {iters.mean(1).round(1)} max {iters.max(1)}")

    def measure_roofline(ctxs, wall_ms, dom=None):
        """Roofline of the dominant kernel class (or of class dom) from the contexts' HIP-event
        brackets (their launches, times and algorithmic bytes summed) over a region of wall_ms."""
        prof = {}
        for kind, name in ((DIE_PROF_PRODUCT, "product"), (DIE_PROF_DOTS, "dots"), (DIE_PROF_AXPY, "axpy"),
                           (DIE_PROF_GEMM, "gemm")):
            cnt = seen = 0
            ms = nbytes = 0.0
            for sv in ctxs:  # summed over the contexts
                c_, s_, m_, b_ = sv.profile_read(kind)
                cnt, seen, ms, nbytes = cnt + c_, seen + s_, ms + m_, nbytes + b_
            if seen:
                prof[name] = dict(timed=cnt, seen=seen, ms=ms, bytes=nbytes)
        est = {k: v["ms"] / max(v["timed"], 1) * v["seen"] for k, v in prof.items()}  # estimated total ms per kind
        if dom is None or dom not in prof:
            dom = max(est, key=est.get)
        p = prof[dom]
        avg_ms = p["ms"] / max(p["timed"], 1)
        work_per_launch = p["bytes"] / max(p["timed"], 1)
        per_kind = {}
        for k, v in prof.items():
            rate = v["bytes"] / max(v["ms"], 1e-9) / 1e6  # GB/s, or GFLOP/s for the GEMM kind
            per_kind[k] = {"launches": v["seen"], "timed": v["timed"], "avg_us": round(1000.0 * v["ms"] / max(v["timed"], 1), 2),
                           ("TFLOPs" if k == "gemm" else "GBs"): round(rate / 1000.0, 2) if k == "gemm" else round(rate, 1),
                           "est_share_of_step": round(est[k] / wall_ms, 3)}
        if dom == "gemm":
            # complex GEMM on the matrix cores: flops against the dense MFMA peak of its precision
            peak = MFMA_PEAK_TFLOPS[16 if args.block_gemm == 16 else args.block_precision]
            achieved = p["bytes"] / (p["ms"] * 1e-3) / 1e12
            # HBM traffic: the operand bytes of the same launches times the measured HBM/algorithmic
            # ratio of the update GEMM (valid only for the solver source the counters were taken on)
            mem_per_launch = sum(sv.profile_mem(DIE_PROF_GEMM) for sv in ctxs) / max(p["timed"], 1)
            src = source_hash("die_te.cpp", "dense.hpp", "ops.hpp", "common.hpp", "kernels_gemm.hip")
            tag = ("block_gemm_update_h16_256" if args.block_gemm == 16 else
                   f"block_gemm_update_c{64 if args.block_precision == 32 else 128}_256")
            traffic = read_traffic(tag, src, mem_per_launch)
            # the bound follows the arithmetic intensity: below the ridge point (peak flops / peak HBM
            # bytes) the GEMM is limited by HBM and is measured in algorithmic bytes per second
            ai = work_per_launch / max(mem_per_launch, 1.0)
            ridge = peak * 1e12 / (HBM_PEAK_GBS * 1e9)
            common = {"kernel": "gemm (block basis update W -= Q H)", "class": "gemm",
                      "traffic": None if traffic is None else int(traffic),
                      "avg_launch_us": round(1000.0 * avg_ms, 2), "algorithmic_flops_per_launch": int(work_per_launch),
                      "algorithmic_bytes_per_launch": int(mem_per_launch), "flops_per_byte": round(ai, 1),
                      "ridge_flops_per_byte": round(ridge, 1), "solver_source_sha256": src, "per_kind": per_kind}
            if ai < ridge:
                gbs = mem_per_launch / (avg_ms * 1e-3) / 1e9
                roofline = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": round(gbs / HBM_PEAK_GBS, 4), "tflops": round(achieved, 2),
                            "mfma_peak_tflops": peak, **common}
            else:
                roofline = {"bound": "mfma", "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
                            "frac": round(achieved / peak, 4), **common}
        else:
            achieved = p["bytes"] / (p["ms"] * 1e-3) / 1e9
            # the kernel file and every header it includes (a traffic summary is only valid for this code)
            src = source_hash(*(("kernels_fft.hip", "fft.hpp", "ops.hpp", "common.hpp") if dom == "product" else
                                ("kernels_krylov.hip", "ops.hpp", "common.hpp")))
            kernel_tag = {"product": "fft_product_c64_256_batched", "dots": "arnoldi_dots_c64_256_batched",
                          "axpy": "arnoldi_axpy_c64_256_batched"}[dom]
            traffic = read_traffic(kernel_tag, src, work_per_launch)
            traffic = None if traffic is None else int(traffic)
            roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "class": dom,
                        "kernel": dom, "avg_launch_us": round(1000.0 * avg_ms, 2),
                        "algorithmic_bytes_per_launch": int(work_per_launch), "kernel_source_sha256": src,
                        "per_kind": per_kind}

        return roofline

    roofline_unc = None
    dom_unc = None
    if concurrent:
        # the contexts' kernels share the chip in the timed call, so the events there also hold
        # other streams' work; one more (untimed) batch of the same block solver on the one
        # four-object context, whose launches have the chip to themselves, gives each class alone
        torch.cuda.synchronize()
        s.profile(3)
        t1 = time.perf_counter()
        _, rc_u, inf_u = s.solve(B, restart=RESTART, max_iters=MAX_ITERS, tol=TOL,
                                 mixed=1 if args.block_precision == 32 else 0,
                                 block=2 if args.block_gemm == 16 else 1, orth=args.block_orth)
        torch.cuda.synchronize()
        wall_u = 1000.0 * (time.perf_counter() - t1)
        s.profile(0)
        roofline_unc = measure_roofline([s], wall_u)
        roofline_unc["batch_ms"] = round(wall_u, 2)
        roofline_unc["converged"] = bool(rc_u == 0 and all(x["rel_res_true"] <= TOL for x in inf_u))
        dom_unc = roofline_unc["class"]
        log(f"roofline, one context, no concurrency: {roofline_unc}")
    # live kernel timings from the library's event brackets over the timed region (for the block
    # solver: the class that dominates when it runs alone)
    roofline = measure_roofline(timed_ctx, ms_per_step * args.steps, dom_unc)
    if concurrent:
        roofline["contended"] = True  # brackets in the timed call overlap the other contexts' kernels
    log(f"roofline: {roofline}")

    out = {
        "metric": "TE solves/s to rel-res 1e-8 (plain vs mixed/batched/learned); matvec % HBM peak",
        "value": round(value, 3), "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 2), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": (("c64 products, f16 block Gram-Schmidt GEMMs (f32 accumulation), c64 CholQR, f64 block least "
                   "squares and refinement") if block and args.block_gemm == 16 else
                  (f"c{64 if args.block_precision == 32 else 128} products and block GEMMs, f64 block least squares "
                   "and refinement") if block else
                  f"f32 products, {'f16' if args.basis == 16 else 'f32'} basis storage, f64 dots/Givens/refinement"),
        "data": "synthetic",
        "config": {"workload": f"random-field objects, 256x256 cells (h = lambda/48), {nobj} objects x "
                               f"{N_ANGLES} TE incidence angles = {nsolve} solves per step",
                   "method": ((f"block GMRES({RESTART}) on A, one block Krylov space per object (its {N_ANGLES} "
                               f"angles), {'complex64' if args.block_precision == 32 else 'complex128'} products and "
                               f"{'one-pass block CGS' if args.block_orth else 'block CGS2'}"
                               f"{' (binary16 planar GEMMs, FP32 accumulation)' if args.block_gemm == 16 else ''}"
                               f" + CholQR GEMMs (a second CholQR pass for ill-conditioned blocks), FP64 block "
                               f"least squares and true-residual restart per cycle, tol {TOL}, zero initial guess, "
                               + (f"all {nsolve} in one die_te_solve_batch call over {nobj} single-object contexts "
                                  f"(a host thread and a stream each)" if concurrent else
                                  f"all {nsolve} in one call of a {nobj}-object context")) if block else
                              (f"batched GMRES({RESTART}) on A, FP32 products, {args.basis}-bit basis storage, "
                               f"{'one-reduction' if args.orth else 'two-pass'} CGS2, FP64 true-residual refinement "
                               f"per cycle, tol {TOL}, zero initial guess, all {nsolve} in one call")),
                   "iters_counted_as": "block steps" if block else "GMRES iterations",
                   "iters_mean": round(float(iters.mean()), 1), "iters_max": int(iters.max()),
                   "products_mean": round(float(prods.mean()), 1),
                   "rel_res_true_max": max(x["rel_res_true"] for x in last), "setup_s": round(setup_s, 3),
                   "fft_variants": {"complex64": timed_ctx[0].fft_plan(N_ANGLES if concurrent else nsolve,
                                                                       torch.complex64),
                                    "complex128": timed_ctx[0].fft_plan(N_ANGLES if concurrent else nsolve,
                                                                        torch.complex128)}},
        "roofline": None,
        "step_kernels": roofline,
    }
    if roofline_unc is not None:
        out["step_kernels_uncontended"] = roofline_unc

    if block and not args.no_variants:
        # the per-rhs batched solver on the same 256 solves, for comparison
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, rc2, inf2 = batch_solve(use_block=False)
        torch.cuda.synchronize()
        t2 = time.perf_counter() - t0
        ok2 = rc2 == 0 and all(x["rel_res_true"] <= TOL for x in inf2)
        out["per_rhs_solver"] = {"value": round(nsolve / t2, 3) if ok2 else 0.0, "unit": "solves/s",
                                 "method": f"per-rhs batched GMRES({RESTART}), one-reduction CGS2, binary16 basis",
                                 "iters_mean": round(float(np.mean([x["iters"] for x in inf2])), 1),
                                 "products_mean": round(float(np.mean([x["products_A"] for x in inf2])), 1)}
        log(f"per-rhs solver: {out['per_rhs_solver']}")

    if not args.no_plain:
        # plain: FP64, one right-hand side per call, same method; angles 0, 16, 32, 48 of each object
        sample = [(o, j) for o in range(nobj) for j in (0, 16, 32, 48)]
        singles = [Solver.from_grid(g, eps[o]) for o in range(nobj)]
        torch.cuda.synchronize()
        its, ok = [], True
        t0 = time.perf_counter()
        for o, j in sample:
            _, rc, inf = singles[o].solve(B[o * N_ANGLES + j], restart=RESTART, max_iters=MAX_ITERS, tol=TOL,
                                          orth=args.orth)
            its.append(inf[0]["iters"])
            ok = ok and rc == 0
        torch.cuda.synchronize()
        tp = time.perf_counter() - t0
        plain = len(sample) / tp if ok else 0.0
        same = [int(iters[o, j]) for o, j in sample]
        out["plain"] = {"value": round(plain, 3), "unit": "solves/s", "dtype": "f64",
                        "sample": "angles 0, 16, 32, 48 of each object (16 of the 256 solves), one call each",
                        "iters": its, "batched_iters_same_solves": same,
                        "ms_per_iter": round(1000.0 * tp / sum(its), 4),
                        "batched_ms_per_solve_iter": round(ms_per_step / float(iters.sum()), 5)}
        out["speedup_vs_plain"] = round(value / plain, 2) if plain > 0 else None
        log(f"plain: {out['plain']}  speedup {out['speedup_vs_plain']}")
        for sv in singles:
            sv.close()

    # product throughput at the batched shape (256 fields, 4 objects, complex64)
    x = torch.randn(nsolve, 2, g.ny, g.nx, dtype=torch.complex64, device="cuda")
    mst = time_matvec(s, x, 10)
    mb = product_model_bytes(g.nx, g.ny, 2 * g.nx, 2 * g.ny, nsolve, 8, nobj)
    out["matvec_batched"] = {"workload": f"{g.nx}x{g.ny} cells, {nobj} objects x {N_ANGLES} fields, complex64",
                             "ms": round(mst, 4), "matvecs_per_s": round(nsolve / mst * 1e3, 1),
                             "model_GBs": round(mb / mst / 1e6, 1),
                             "frac_hbm": round(mb / mst / 1e6 / HBM_PEAK_GBS, 4)}
    log(f"batched-shape product: {out['matvec_batched']}")
    del x

    # the roofline of the product kernels at the largest class of the batched workload (1024^2
    # cells, 64 fields, complex64), where each pass's working set is far beyond the last-level cache
    out["roofline"] = product_roofline()
    log(f"roofline (product at 1024^2 x 64): {out['roofline']}")

    if not args.no_configured_deflation:
        # the batched configuration's deflation (k = 16 per object) on the headline batch, with the
        # headline's block solver (capped), beside the undeflated headline
        t0 = time.perf_counter()
        sds = [Solver.from_grid(g, eps[o], deflate_k=16, seed=1) for o in range(nobj)]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        res_d, rc_d = Solver.solve_batch(sds, B_obj, restart=RESTART, max_iters=1500, tol=TOL, mixed=1, block=2,
                                         orth=args.block_orth)
        torch.cuda.synchronize()
        inf = [x for _, i in res_d for x in i]
        it_d = np.array([x["iters"] for x in inf])
        out["configured_deflation_k16"] = {
            "method": "the headline's block solver on A P^-1, k = 16 per object, capped at 1500 block steps",
            "converged": int(sum(x["status"] == 0 for x in inf)), "of": nsolve,
            "iters_mean": round(float(it_d.mean()), 1), "iters_max": int(it_d.max()),
            "iters_mean_undeflated": round(float(iters.mean()), 1),
            "worst_rel_res": max(x["rel_res_true"] for x in inf), "setup_s": round(t1 - t0, 2),
            "s": round(time.perf_counter() - t1, 2)}
        log(f"configured deflation: {out['configured_deflation_k16']}")
        for sv in sds:
            sv.close()

    if not args.no_variants:
        # the paper's four systems on the hard cylinder, its 128^2 analog and Table 2's squares
        out["method_variants"] = method_variants()

    if not args.no_learned:
        out["learned"] = learned_leg(lambda x0s: batch_solve(x0s=x0s), timed_ctx, B_obj if concurrent else [B],
                                     args.steps, nsolve, value, iters,
                                     out["plain"]["value"] if "plain" in out else None)
        log(f"learned: {out['learned']}")

    if args.uneven:
        # the headline's contexts hold block buffers the 1024^2 class needs
        for sv in per_obj:
            sv.close()
        s.close()
        torch.cuda.empty_cache()
        out["uneven"] = uneven_run([int(v) for v in args.uneven.split(",")], args, deflate_k=args.uneven_deflate,
                                   budget_s=args.uneven_budget or None)

    if not args.no_cpu_baseline:
        log("timing the CPU oracle (direct-sum products, dense solves) ...")
        out["cpu_baseline"] = cpu_baseline(g, eps[0], N_ANGLES)
        log(f"cpu baseline: {out['cpu_baseline']}")
    s.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
