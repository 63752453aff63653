"""Benchmark: time-to-solution of PP-GMRES and p(A)v bandwidth on one MI355X.

Workload (the one the headline metric is quoted on): 3-D convection-diffusion
-Lap u + 10 (u_x + u_y + u_z), 7-point finite differences on a 128^3 grid
(n = 2,097,152, nnz = 14,581,760), b ~ N(0,1) normalised, polynomial of
degree 40 from GMRES(40) on a seeded N(0,1) start vector with roots added
for stability, PP-GMRES(50) to a true relative residual of 1e-8.

One step = polynomial setup + solve (the whole hot path) with the p/phi
chains and Krylov vectors in FP32 inside FP64 iterative refinement. The
plain FP64 form is timed beside it. Inputs are resident in HBM before the
timed region. Prints one JSON line.

More legs are reported beside the headline (skip with --no-extras): the
random sparse workload (n = 1e6) in FP64/FP32/BF16, the chain step on the
same stencil at 256^3 (long launches: the kernel's streaming rate),
differentiation
through the solve on a 1024^2 2-D system (forward + adjoint), the batched
solve of 256 systems x 4 right-hand sides against loops of single solves,
and the paper's own synthetic rows run beside its printed figures.
"""

import argparse
import functools
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time-to-solution @1e-8 rel. residual; p(A)v achieved HBM GB/s (FP32 vs FP64)"
HBM_PEAK_GBPS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def step_bytes(n, nnz, s_val, s_vec):
    """Algorithmic bytes of one chain step: CSR read once, input read once, output written once."""
    return nnz * (s_val + 4) + 4 * (n + 1) + 2 * n * s_vec


# HBM traffic of the chain kernel, from rocprofv3 --pmc (FETCH_SIZE, WRITE_SIZE)
# runs of ``bench.py --traffic-probe``, kept with the command that made it.
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "traffic_chain_step_convdiff3d_128.md")
KERNEL_SOURCES = ("kernels.hip", "kernels.h", "devutil.h")
COPY_BYTES = 1 << 30  # calibration copy: 1 GiB read + 1 GiB written


def code_text(src):
    """C++ source without comments and blank lines, each line stripped, so
    that the hash below changes with the code and not with its comments."""
    import re

    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    out = []
    for line in src.splitlines():
        line = re.sub(r"//.*$", "", line).strip()
        if line:
            out.append(line)
    return "\n".join(out)


def kernel_source_hash():
    """sha256 over the code (comments dropped) the chain kernels are compiled from."""
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1911_07065_amd", "csrc", f), encoding="utf-8") as fh:
            h.update(code_text(fh.read()).encode())
    return h.hexdigest()


def chain_kernel_name(variant):
    """The FP32 chain-step kernel behind a tuned variant name."""
    v = variant or "?"
    if v.startswith("sell64d16"):
        return f"k_chain_sell<float,float,...,short> ({v}: sliced-ELL, 16-bit column offsets, fused chain update)"
    if v.startswith("sell"):
        return f"k_chain_sell<float,float,...,int> ({v}: sliced-ELL SpMV fused with the chain update)"
    if v == "diap":
        return ("k_chain_diap<float,float,nd> (diap: diagonal format with one byte per row naming its pattern "
                "among the matrix's distinct rows, fused chain update)")
    if v.startswith("diac"):
        return (f"k_chain_diac<float,float,nd,rows> ({v}: diagonal format with 1-byte codes into the matrix's "
                "distinct values, fused chain update)")
    if v == "dia1":
        return "k_chain_dia_nd<float,float,nd> (dia1: diagonal format, one row per lane, fused chain update)"
    if v.startswith("dia"):
        return f"k_chain_dia<float,float,...> ({v}: diagonal format, fused chain update)"
    if v == "box":
        return ("k_chain_box<float,float,7> (box: constant-coefficient box stencil, no per-row matrix data, "
                "4 points of a grid line per lane, fused chain update)")
    if v == "box/tile2":
        return ("k_chain_boxt<float,float,16,4,128,1024> (two chain steps per launch on tiles of 16 x 4 whole "
                "grid lines, 1024 threads, the input and the first step staged in LDS)")
    if v.startswith("csort"):
        wide = "true" if v == "csort2" else "false"
        return (f"k_chain_cs_tiles<float,float,{wide}> + k_chain_cs_finish ({v}: (8192-row block, column band) "
                f"tiles whose entries are sorted by column, {v[-1]} partial row sums, then the fused chain update)")
    return f"chain step, variant {v}"


def recorded_traffic(prec, variant, remap):
    """Measured HBM bytes per launch for (prec, variant, remap), or None when
    there is no record, it is for other kernel sources, or other variants."""
    try:
        with open(TRAFFIC_RECORD) as fh:
            line = next(l for l in fh if l.startswith("TRAFFIC_RECORD "))
        rec = json.loads(line[len("TRAFFIC_RECORD "):])
    except (OSError, StopIteration, ValueError):
        return None
    if rec.get("source_sha256") != kernel_source_hash():
        return None
    for e in rec.get("kernels", []):
        # remap -1: launches in the tuned workgroup order (two-step tiles)
        if e["prec"] == prec and e["variant"] == variant and e["remap"] in (remap, -1):
            return e
    return None


def traffic_probe(pp, torch, np, M, n):
    """Launch sequence for the counter runs: a plain copy of COPY_BYTES (to
    calibrate FETCH_SIZE and WRITE_SIZE), then for each sliced-ELL,
    diagonal-format and box variant, precision and XCD order (remap 1, then
    0) 4 phi applications of an 8-root real polynomial (32 launches of
    exactly one chain step each: the input read and gathered, the output
    written), then, where they apply, the same with two steps per launch on
    whole grid lines ("box/tile2": 16 launches, each reading its input once
    and writing its second step's result)."""
    x = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    del x, y
    log("copy", COPY_BYTES, "bytes x3")
    poly = pp.poly_from_roots(np.linspace(2.0, 11.0, 8), keep_order=True)
    names = [pp.chain_variant_name(v) for v in range(pp.N_CHAIN_VARIANTS)]
    for prec, dt in (("fp32", torch.float32), ("fp64", torch.float64)):
        v = torch.as_tensor(np.random.default_rng(5).standard_normal(n), device="cuda").to(dt)
        out = torch.empty_like(v)
        for vi, name in enumerate(names):
            if not (name.startswith("sell") or name.startswith("dia") or name == "box"):
                continue
            for remap in (1, 0):  # the counter summary splits each kernel's dispatches in this order
                try:
                    M.set_variant(prec, vi, remap)
                except Exception as exc:  # a copy this matrix does not have
                    log("probe", prec, name, "skipped:", exc)
                    break
                for _ in range(4):
                    pp.apply(poly, M, v, "phi", out=out)
                torch.cuda.synchronize()
                log("probe", prec, name, f"remap {remap}: 32 launches")
        try:
            M.set_variant(prec, names.index("box"), 1)
            M.set_march_shape(1, prec)
        except Exception as exc:
            log("probe", prec, "box/tile2 skipped:", exc)
            continue
        for _ in range(4):
            pp.apply(poly, M, v, "phi", out=out)
        torch.cuda.synchronize()
        log("probe", prec, "box/tile2: 16 launches")
    log("kernel sources sha256", kernel_source_hash())


def chain_rate(pp, torch, np, M, poly, prec, dt, reps, kind="phi", n=None):
    """Time reps back-to-back applications of poly on M (HIP events on the
    stream the library launches on) and return the time per launch and the
    rate of the bytes the launches must move by their definition
    (pp_chain_bytes)."""
    stream = torch.cuda.current_stream()
    v = torch.as_tensor(np.random.default_rng(5).standard_normal(n or M.n), device="cuda").to(dt)
    y = torch.empty_like(v)
    for _ in range(2):
        pp.apply(poly, M, v, kind, out=y)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        pp.apply(poly, M, v, kind, out=y)
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    by, launches = pp.chain_bytes(poly, M, kind, prec)
    del v, y
    return {"variant": M.variant(prec)[0], "ms": ms, "launches": launches, "launch_us": ms * 1e3 / launches,
            "bytes": by, "bytes_per_launch": by / launches, "GBps": by / (ms * 1e-3) / 1e9,
            "frac": by / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS}


def launch_floor_us(pp, torch, blocks, threads=256, reps=200):
    """Time per launch of back-to-back empty kernels of `blocks` workgroups
    of `threads` threads (pp_launch_floor), HIP events on the stream they run
    on."""
    stream = torch.cuda.current_stream()
    pp.launch_floor(20, blocks, threads)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    pp.launch_floor(reps, blocks, threads)
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) * 1e3 / reps


def scale_leg(pp, torch, np, N=256, nroots=16, reps=10):
    """The chain step on the 3-D convection-diffusion matrix at N^3 = 256^3
    (n = 16.8 M), where one launch streams long enough that its ramp and
    drain are small next to the transfer: a phi polynomial of 16 real roots
    timed with HIP events, FP32 and FP64, with the autotuner's choice (one
    step per launch, or two on whole grid lines); rates from the bytes the
    launches must move (pp_chain_bytes). step_us is per chain step, launch_us
    per launch."""
    from workloads import convdiff3d

    log("scale leg: generating", N)
    csr = convdiff3d(N, 10.0, 10.0, 10.0)
    n, nnz = csr.n, csr.nnz
    M = pp.Matrix.from_csr(csr)
    del csr
    poly = pp.poly_from_roots(np.linspace(2.0, 11.0, nroots), keep_order=True)
    out = {"workload": f"3-D convection-diffusion {N}^3 (n={n}, nnz={nnz}), phi(A)v of {nroots} real roots"}
    for prec, dt, sx in (("fp32", torch.float32, 4), ("fp64", torch.float64, 8)):
        M.tune(prec)
        r = chain_rate(pp, torch, np, M, poly, prec, dt, reps)
        g = M.march(prec)[0]
        fused = "/tile2" if g == 2 and M.march_shape(prec) == 1 else (f"/march{g}" if g >= 2 else "")
        step_us = r["ms"] * 1e3 / nroots
        out[prec] = {"variant": r["variant"] + fused, "step_us": round(step_us, 3),
                     "launch_us": round(r["launch_us"], 3), "launches": r["launches"],
                     "bytes_per_launch": int(r["bytes_per_launch"]), "GBps": round(r["GBps"], 1),
                     "frac": round(r["frac"], 4),
                     "csr_equiv_GBps": round(step_bytes(n, nnz, sx, sx) / (step_us * 1e-6) / 1e9, 1)}
        log("scale leg", prec, out[prec]["variant"], f"{step_us:.2f} us/step", f"{r['launch_us']:.2f} us/launch",
            f"{r['GBps']:.0f} GB/s own bytes")
    del M
    torch.cuda.empty_cache()
    return out


def out_of_mall_leg(pp, torch, np, reps=5, nroots=8):
    """One point per chain-kernel family whose working set is well above the
    256 MB MALL, so each launch streams from HBM: the pattern-coded diagonal
    kernel (diapv) at 384^3 (FP32: input + output + pattern bytes = 509 MB
    per step), the constant-coefficient box kernel at 384^3 (input + output =
    453 MB), the sliced-ELL kernel (sell64) and the CSR row-tile kernel
    (tile8x1) at 256^3 (FP32: 1.08 GB of matrix and vectors per step). Each
    is forced (no tuning), phi(A)v of 8 real roots, HIP events, bytes from
    pp_chain_bytes; FP32 and FP64."""
    from workloads import convdiff3d

    out = {}
    names = [pp.chain_variant_name(k) for k in range(pp.N_CHAIN_VARIANTS)]
    poly = pp.poly_from_roots(np.linspace(2.0, 11.0, nroots), keep_order=True)
    for N, variants in ((384, ("diapv", "box")), (256, ("sell64", "tile8x1"))):
        log("out-of-MALL leg: generating", N)
        csr = convdiff3d(N, 10.0, 10.0, 10.0)
        n, nnz = csr.n, csr.nnz
        log("out-of-MALL leg: matrix handle", N, "nnz", nnz)
        M = pp.Matrix.from_csr(csr)
        del csr
        for v in variants:
            for prec, dt in (("fp32", torch.float32), ("fp64", torch.float64)):
                M.set_variant(prec, names.index(v), 1)
                r = chain_rate(pp, torch, np, M, poly, prec, dt, reps)
                key = f"{v}_{N}_{prec}"
                out[key] = {"workload": f"3-D convection-diffusion {N}^3 (n={n}, nnz={nnz})", "kernel": v,
                            "step_us": round(r["launch_us"], 3), "bytes_per_step": int(r["bytes_per_launch"]),
                            "GBps": round(r["GBps"], 1), "frac": round(r["frac"], 4)}
                log("out-of-MALL", key, f"{r['launch_us']:.1f} us/step", f"{r['GBps']:.0f} GB/s",
                    f"frac {r['frac']:.3f}")
        del M
        torch.cuda.empty_cache()
    return out


def adjoint_leg(pp, torch, np):
    """Differentiation through the solve: loss 0.5 ||x(theta, b) - x_t||^2 on
    the 2-D convection-diffusion 1024^2 system whose convection coefficient
    theta = 20 is a leaf tensor; degree 50, GMRES(50), tol 1e-12, FP64.
    Timed: polynomial setup, forward solve and adjoint solve (same roots on
    the transposed pattern), after one untimed pass."""
    from workloads import convdiff2d_parts, rhs, start_vector

    N, theta0 = 1024, 20.0
    A0, dval = convdiff2d_parts(N)
    n = N * N
    M = pp.Matrix.from_csr(A0)
    base = torch.as_tensor(A0.val, device="cuda")
    dirv = torch.as_tensor(dval, device="cuda")
    bd = torch.as_tensor(rhs(n, 1), device="cuda")
    xt = torch.as_tensor(np.random.default_rng(3).standard_normal(n), device="cuda")
    v0 = torch.as_tensor(start_vector(n, 2), device="cuda")

    def once():
        M.set_values(base + theta0 * dirv)
        poly = pp.setup(M, v0, 50)
        th = torch.tensor(theta0, dtype=torch.float64, device="cuda", requires_grad=True)
        bt = bd.clone().requires_grad_(True)
        x = pp.pp_solve_fn(base + th * dirv, bt, M, poly, tol=1e-12, m=50, inner="fp64")
        loss = 0.5 * torch.sum((x - xt) ** 2)
        loss.backward()
        return float(th.grad), float(torch.linalg.norm(bt.grad))

    once()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g, gb = once()
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    log("adjoint", f"{t * 1e3:.1f} ms", "dL/dtheta", g)
    At = getattr(M, "_t", None)  # the transpose handle the adjoint solve ran on (kept across calls)

    def chain_of(H):
        fused, _, us_pair = H.pair_steps("fp64")
        g, cz, us_m = H.march("fp64")
        return {"variant": H.variant("fp64")[0], "two_steps_per_launch": fused, "two_step_launch_us": round(us_pair, 3),
                "march_steps_per_launch": g, "march_launch_us": round(us_m, 3)}

    return {"workload": f"2-D convection-diffusion {N}^2 (n={n}, nnz={A0.nnz}), theta=20 leaf, "
                        "PP(50)-GMRES(50) to 1e-12 FP64, forward + adjoint",
            "time_s": round(t, 6), "dL_dtheta": g, "norm_dL_db": gb,
            "note": "timed after one untimed pass: the transpose handle (pattern, copies, tuning) is made in that "
                    "pass and reused, its values gathered from the new A",
            "forward_chain_fp64": chain_of(M), "adjoint_chain_fp64": chain_of(At) if At is not None else None}


def random_sparse_leg(pp, torch, np, reps=5):
    """Random sparse workload: n = 1e6, 16 distinct off-diagonal columns per
    row plus the diagonal, diagonally dominant, degree 100 with added roots,
    GMRES(30), tol 1e-8. Time-to-solution (setup included) in FP64, FP32 and
    BF16 storage (the latter two with an FP32-basis setup), and p(A)v per
    chain launch with its CSR algorithmic rate."""
    from workloads import randsparse, rhs, start_vector

    csr = randsparse(1_000_000, 16, seed=7)
    n, nnz = csr.n, csr.nnz
    A = csr.to_scipy()
    b = rhs(n, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    M = pp.Matrix.from_csr(csr)
    torch.cuda.synchronize()
    t_create = time.perf_counter() - t0
    bd = torch.as_tensor(b, device="cuda")
    v0 = torch.as_tensor(start_vector(n, 2), device="cuda")
    out = {"workload": f"random sparse n={n}, nnz={nnz} (16 random columns + diagonal, dominance 1.05), "
                       "PP(100+added)-GMRES(30) to 1e-8, setup included",
           "matrix_create_s": round(t_create, 3)}
    log("random sparse matrix handle (all copies, column-sorted tiles included)", f"{t_create:.3f} s")
    stream = torch.cuda.current_stream()
    poly = None
    for inner in ("fp64", "fp32", "bf16"):
        # the reduced-precision forms take the polynomial from an FP32-basis setup
        basis = "fp64" if inner == "fp64" else "fp32"
        poly = pp.setup(M, v0, 100, basis=basis)
        pp.solve(poly, M, bd, tol=1e-8, m=30, inner=inner)  # warm-up (tuning)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        poly = pp.setup(M, v0, 100, basis=basis)
        x, info = pp.solve(poly, M, bd, tol=1e-8, m=30, inner=inner)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        rel = float(np.linalg.norm(b - A @ x.cpu().numpy()) / np.linalg.norm(b))
        out[f"time_to_solution_s_{inner}"] = round(t, 6)
        out[f"relres_{inner}"] = rel
        out[f"cycles_{inner}"] = info["cycles"]
        out[f"setup_basis_{inner}"] = basis
        log("random sparse", inner, f"{t * 1e3:.1f} ms", "relres", rel, "cycles", info["cycles"], "setup basis", basis)
    out["d_eff"] = poly.d_eff
    for prec, dt, sv, sx in (("fp32", torch.float32, 4, 4), ("fp64", torch.float64, 8, 8),
                             ("bf16", torch.bfloat16, 4, 2)):
        r = chain_rate(pp, torch, np, M, poly, prec, dt, reps)
        us = r["ms"] * 1e3 / poly.d_eff  # per chain step (a banded step is one launch per band)
        out[f"chain_step_us_{prec}"] = round(us, 3)
        out[f"chain_step_bytes_{prec}"] = int(r["bytes"] / poly.d_eff)
        out[f"chain_step_GBps_{prec}"] = round(r["GBps"], 1)
        out[f"chain_step_frac_{prec}"] = round(r["frac"], 4)
        out[f"chain_step_csr_equiv_GBps_{prec}"] = round(step_bytes(n, nnz, sv, sx) / (us * 1e-6) / 1e9, 1)
        out[f"chain_variant_{prec}"] = r["variant"]
        log("random sparse phi step", prec, r["variant"], f"{us:.2f} us", out[f"chain_step_GBps_{prec}"], "GB/s",
            "frac", out[f"chain_step_frac_{prec}"])
    return out


def preconditioned_leg(pp, torch, np, N=512, bs=4, d=10):
    """Composition with a right preconditioner (eqs. 1.3-1.4): the 2-D
    convection-diffusion matrix on an N x N grid times a block-diagonal
    mixing of 4 x 4 blocks (two decades either way), solved to 1e-8 with
    block-Jacobi (B = A M^{-1} formed once from A's inverted diagonal blocks;
    the polynomial is built for B) and FP32 inner cycles. The same degree on
    A itself is run with a cap of 30 cycles."""
    from workloads import convdiff2d_blockmixed, rhs, start_vector

    csr = convdiff2d_blockmixed(N, 5.0, bs, 2.0)
    n = csr.n
    b = torch.as_tensor(rhs(n, 1), device="cuda")
    v0 = torch.as_tensor(start_vector(n, 2), device="cuda")
    A = pp.Matrix.from_csr(csr)
    out = {"workload": f"2-D convection-diffusion {N}^2 times 4x4 block mixing (n={n}, nnz={csr.nnz}), "
                       f"PP({d})-GMRES(50) to 1e-8, FP32 inner / FP64 outer"}
    for rep in range(2):  # the first pass builds and tunes; the second is timed
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        B = A.block_jacobi(bs)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        x, info = pp.solve(pp.setup(B, v0, d), B, b, tol=1e-8, m=50, inner="fp32")
        torch.cuda.synchronize()
        t2 = time.perf_counter()
    out.update(block_jacobi_build_s=round(t1 - t0, 6), time_to_solution_s=round(t2 - t1, 6),
               converged=bool(info["converged"]), cycles=info["cycles"], relres=info["relres"],
               nnz_b=int(B.nnz))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, info0 = pp.solve(pp.setup(A, v0, d), A, b, tol=1e-8, m=50, max_cycles=30, inner="fp32")
    torch.cuda.synchronize()
    out.update(plain_converged=bool(info0["converged"]), plain_cycles=info0["cycles"],
               plain_relres=info0["relres"], plain_time_s=round(time.perf_counter() - t0, 6))
    log("block-Jacobi", f"{out['time_to_solution_s'] * 1e3:.1f} ms", "cycles", out["cycles"],
        "build", f"{out['block_jacobi_build_s'] * 1e3:.0f} ms", "plain converged", out["plain_converged"],
        "relres", out["plain_relres"])
    return out


def paper_context_leg(pp, torch, np):
    """The paper's synthetic rows run on the GPU beside its printed counts and
    times (MATLAB on an Intel i7-6700, FP64, MGS): Table 3.6 (2-D
    convection-diffusion, n = 40000, PP(50)-GMRES(50), alpha = beta = gamma = 0),
    Table 4.1 (diag(i^2/n), n = 20000, d = 256, GMRES(50), tol 1e-10) and
    Table 3.4 / Example 13 (biharmonic, n = 40000, d = 200 and the 40 x 40
    double polynomial; true residual 2e-10 for the paper's shortcut 1e-10).
    FP64 throughout."""
    from workloads import biharmonic2d, convdiff2d, diag_squares, rhs, start_vector

    rows = []

    def run(name, csr, d, tol, paper, double=None):
        M = pp.Matrix.from_csr(csr)
        bd = torch.as_tensor(rhs(csr.n, 1), device="cuda")
        v0 = torch.as_tensor(start_vector(csr.n, 2), device="cuda")
        for timed in (False, True):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            p = pp.setup(M, v0, d)
            setup_mv, setup_dots = p.setup_info["mvps"], p.setup_info["dots"]
            if double:
                p2 = pp.setup_double(M, p, v0, double)
                setup_mv += p2.setup_info["mvps"]
                setup_dots += p2.setup_info["dots"]
                p = p2
            x, info = pp.solve(p, M, bd, tol=tol, m=50, max_cycles=20000, inner="fp64", stall_cycles=0)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
        rows.append({"case": name, "cycles": info["cycles"], "mvps": info["mvps"] + setup_mv,
                     "dots": info["dots"] + setup_dots, "time_s": round(t, 4), "converged": info["converged"],
                     "paper": paper})
        log("paper context", rows[-1])

    run("Table 3.6 row 1: 2-D conv.-diff. n=40000, PP(50)-GMRES(50), tol 1e-8", convdiff2d(200, 0.0), 50, 1e-8,
        {"mvps": 1051, "time_s": 0.95})
    run("Table 4.1: diag(i^2/n) n=20000, PP(256)-GMRES(50), tol 1e-10", diag_squares(20000), 256, 1e-10,
        {"cycles": 43, "mvps": 542000, "dots": 89000, "time_s": 40.9})
    bh = biharmonic2d(200)
    run("Table 3.4: biharmonic n=40000, PP(200)-GMRES(50), true residual 2e-10", bh, 200, 2e-10,
        {"cycles": 11, "mvps": 105000, "dots": 33900, "time_s": 54.9})
    run("Table 6.1: biharmonic n=40000, double 40x40, GMRES(50), true residual 2e-10", bh, 40, 2e-10,
        {"cycles": 1, "mvps": 75300, "dots": 2760, "time_s": 35.8}, double=40)
    return {"hardware_of_paper": "MATLAB, Dell Optiplex, Intel i7-6700, FP64, modified Gram-Schmidt",
            "ours": "one MI355X, FP64, CGS2 (dots count both passes)", "rows": rows}


def batched_leg(pp, torch, np, loop_every=16, orth="delayed", graph_steps=5):
    """Batched solve: 256 2-D convection-diffusion systems (sides U{64..512},
    coefficient U[0,50)), 4 right-hand sides each, degree 20, GMRES(50),
    FP32 inner / FP64 outer, tol 1e-8 (setup + solve), against a loop of
    single-system solves timed on every 16th system (matrix handle made and
    tuned outside the timing) and scaled to the batch."""
    from workloads import batched_convdiff_specs, convdiff2d, rhs, start_vector

    specs = batched_convdiff_specs()
    csrs = [convdiff2d(N, a) for (N, a, _, _) in specs]
    B = pp.Batch(csrs)
    B.set_orth(orth)
    v0 = torch.as_tensor(np.concatenate([start_vector(N * N, s2) for (N, _, _, s2) in specs]), device="cuda")
    brs = [rhs(N * N, s1, count=4) for (N, _, s1, _) in specs]
    bd = B.interleave(np.concatenate(brs, axis=1))
    # the batched autotuner (chain kernel shape per precision) runs outside the timing
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tuned = {prec: B.tune(4, prec) for prec in ("fp32", "fp64")}
    torch.cuda.synchronize()
    t_tune = time.perf_counter() - t0
    log("batched tuner", tuned, f"{t_tune * 1e3:.1f} ms")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    polys = B.setup(v0, 20)
    x, infos = B.solve(polys, bd, 4, tol=1e-8, m=50, inner="fp32", graph_steps=graph_steps)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    ok = all(i["converged"] for i in infos)
    worst = max(i["relres"] for i in infos)
    log("batched", f"{t_batch:.3f} s", "converged", ok, "worst relres", worst)
    t_loop, t_loop64, sub = 0.0, 0.0, list(range(0, len(csrs), loop_every))
    for s in sub:
        M = pp.Matrix.from_csr(csrs[s])
        M.tune("fp32")
        M.tune("fp64")
        bs = [torch.as_tensor(brs[s][r], device="cuda") for r in range(4)]
        v0s = torch.as_tensor(start_vector(csrs[s].n, specs[s][3]), device="cuda")
        for inner in ("fp32", "fp64"):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            poly = pp.setup(M, v0s, 20)
            for r in range(4):
                pp.solve(poly, M, bs[r], tol=1e-8, m=50, inner=inner)
            torch.cuda.synchronize()
            if inner == "fp32":
                t_loop += time.perf_counter() - t1
            else:
                t_loop64 += time.perf_counter() - t1
    t_loop *= len(csrs) / len(sub)
    t_loop64 *= len(csrs) / len(sub)
    log("loop of single solves (scaled)", f"{t_loop:.3f} s", "plain FP64", f"{t_loop64:.3f} s")
    return {"workload": f"256 x 2-D convection-diffusion (sum n={B.n}, nnz={B.nnz}), 4 RHS each, PP(20)-GMRES(50) "
                        "to 1e-8, FP32 inner / FP64 outer, setup included",
            "time_s": round(t_batch, 6), "all_converged": ok, "worst_relres": worst,
            "loop_time_s": round(t_loop, 6), "loop_fp64_time_s": round(t_loop64, 6),
            "loop_sample": f"every {loop_every}th system, scaled, handles made and tuned outside the timing",
            "chain_shape": {prec: {"format": t[0], "slices_per_wave": t[1], "xcd_order": t[2], "step_us": round(t[3], 2)}
                            for prec, t in tuned.items()},
            "tune_s": round(t_tune, 6),
            "cycle": f"device Givens per pair; HIP graphs of {graph_steps} Arnoldi steps, one host check between them",
            "orth": orth,
            "speedup_vs_loop": round(t_loop / t_batch, 3), "speedup_vs_fp64_loop": round(t_loop64 / t_batch, 3)}


def host_cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform

    return platform.processor() or "unknown"


def cpu_baseline(csr, b, v0, d, m, reps=3, cap_s=100.0, gpu_x=None):
    """The FP64 oracle's full time-to-solution on the host (polynomial setup by
    GMRES(d) with modified Gram-Schmidt, Leja order and added roots, then
    PP(d)-GMRES(m) to 1e-8, as the paper times it): the median of up to
    `reps` runs, fewer when the runs so far took more than cap_s. gpu_x:
    {form: x} of the GPU solutions, each compared with the oracle's x."""
    import numpy as np

    from oracle import roots, solver

    try:
        from threadpoolctl import threadpool_info

        threads = max([1] + [i.get("num_threads", 1) for i in threadpool_info()])
    except Exception:
        threads = os.cpu_count() or 1
    A = csr.to_scipy()
    times, info = [], None
    t_all = time.perf_counter()
    while len(times) < reps:
        t0 = time.perf_counter()
        P = roots.setup(A, v0, d)
        x, info = solver.pp_gmres(A, b, P.units, m=m, tol=1e-8, setup_mvps=P.d)
        times.append(time.perf_counter() - t0)
        log("oracle full solve on the host", f"{times[-1]:.1f} s", "cycles", info.cycles, "relres", info.relres)
        if time.perf_counter() - t_all > cap_s:
            break
    rel = float(np.linalg.norm(b - A @ x) / np.linalg.norm(b))
    xerr = {k: float(np.linalg.norm(v - x) / np.linalg.norm(x)) for k, v in (gpu_x or {}).items()}
    return {
        "x_err_vs_oracle": xerr,
        "value": float(np.median(times)),
        "unit": "s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": (f"full FP64 numpy/scipy oracle time-to-solution of the same workload: GMRES({d}) setup with "
                   f"modified Gram-Schmidt, Leja order and added roots, then PP({P.d}+{P.n_added})-GMRES({m}) to "
                   f"1e-8 ({info.cycles} cycles, {info.iters} Arnoldi steps, relres {rel:.2e}); median of "
                   f"{len(times)} run(s): " + ", ".join(f"{t:.2f}" for t in times) + " s"),
        "runs_s": [round(t, 3) for t in times],
        "cpu_model": host_cpu_model(),
        "os_cpu_count": os.cpu_count(),
        "blas_threads": int(threads),
        "OPENBLAS_NUM_THREADS": os.environ.get("OPENBLAS_NUM_THREADS"),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--grid", type=int, default=128)
    ap.add_argument("--degree", type=int, default=40)
    ap.add_argument("--m", type=int, default=50)
    ap.add_argument("--pav-reps", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-reps", type=int, default=3, help="oracle runs on the host (median; capped at ~100 s)")
    ap.add_argument("--setup-basis", default="fp32", choices=["fp32", "fp64"],
                    help="Krylov vector storage of the FP32 form's polynomial setup (the FP64 form's is fp64)")
    ap.add_argument("--batch-graph-steps", type=int, default=5,
                    help="Arnoldi steps per captured segment of a batched cycle (one host check per segment)")
    ap.add_argument("--batch-orth", default="delayed", choices=["delayed", "cgs2"],
                    help="orthogonalisation of the batched cycles (delayed: two basis sweeps per step)")
    ap.add_argument("--chain-variant", default=None,
                    help="pin the chain kernel instead of autotuning, remap on: a variant name for both precisions "
                         "(e.g. diac) or fp32=<v>,fp64=<w>; <v>/tile2 adds two steps per launch on whole grid "
                         "lines. Used to profile what an unprofiled run picks (the tracer's launch overhead "
                         "shifts the tuner's choices)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the differentiation and batched legs")
    ap.add_argument("--leg", default=None,
                    choices=["random_sparse", "chain_step_256", "adjoint", "batched", "preconditioned",
                             "paper_context", "out_of_mall"],
                    help="run only this side workload and print its JSON (for profiling one workload)")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="only run the launch sequence the rocprofv3 counter runs read (no JSON line)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): this library has no multi-GPU path. "
              "Across GPUs the rows would split into blocks, with one halo exchange per chain step and one "
              "small all-reduce per Gram-Schmidt pass.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1911_07065_amd.api as pp
    from workloads import convdiff3d, rhs, start_vector

    assert torch.cuda.is_available(), "bench.py needs a ROCm GPU"
    if args.leg:
        legs = {"random_sparse": random_sparse_leg, "chain_step_256": scale_leg, "adjoint": adjoint_leg,
                "batched": batched_leg, "preconditioned": preconditioned_leg, "paper_context": paper_context_leg,
                "out_of_mall": out_of_mall_leg}
        fn = legs[args.leg]
        if args.leg == "batched":
            fn = functools.partial(batched_leg, orth=args.batch_orth, graph_steps=args.batch_graph_steps)
        print(json.dumps({args.leg: fn(pp, torch, np)}))
        return
    N, d, m, tol = args.grid, args.degree, args.m, 1e-8
    log("generating workload", N)
    csr = convdiff3d(N, 10.0, 10.0, 10.0)
    n, nnz = csr.n, csr.nnz
    b = rhs(n, 1)
    v0 = start_vector(n, 2)
    # the handle's one-time costs, outside the timed steps: the CSR arrays are
    # uploaded first, then pp_matrix_create (host analysis of the pattern and
    # the library's storage copies) and the autotuner for both precisions
    rp_d = torch.as_tensor(csr.rowptr, device="cuda")
    ci_d = torch.as_tensor(csr.colind, device="cuda")
    va_d = torch.as_tensor(csr.val, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    M = pp.Matrix(rp_d, ci_d, va_d)
    torch.cuda.synchronize()
    t_create = time.perf_counter() - t0
    t_tune = 0.0
    if not args.chain_variant:
        t0 = time.perf_counter()
        M.tune("fp32")
        M.tune("fp64")
        torch.cuda.synchronize()
        t_tune = time.perf_counter() - t0
    log("matrix handle", f"create {t_create * 1e3:.1f} ms", f"tune {t_tune * 1e3:.1f} ms")
    if args.chain_variant:
        # "v" for both precisions, or "fp32=v,fp64=w"; "v/tile2": two steps
        # per launch on whole grid lines after single steps of v
        names = [pp.chain_variant_name(k) for k in range(pp.N_CHAIN_VARIANTS)]
        spec = {}
        for part in args.chain_variant.split(","):
            if "=" in part:
                prec, v = part.split("=", 1)
                spec[prec] = v
            else:
                spec["fp32"] = spec["fp64"] = part
        for prec, v in spec.items():
            M.set_variant(prec, names.index(v.split("/")[0]), 1)
            if v.endswith("/tile2"):
                M.set_march_shape(1, prec)
        log("chain variant pinned:", spec)
    bd = torch.as_tensor(b, device="cuda")
    v0d = torch.as_tensor(v0, device="cuda")
    torch.cuda.synchronize()
    if args.traffic_probe:
        traffic_probe(pp, torch, np, M, n)
        return

    def step(inner):
        poly = pp.setup(M, v0d, d, basis=args.setup_basis if inner == "fp32" else "fp64")
        x, info = pp.solve(poly, M, bd, tol=tol, m=m, inner=inner)
        return poly, x, info

    res = {}
    for inner in ("fp32", "fp64"):
        for _ in range(args.warmup):
            step(inner)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            poly, x, info = step(inner)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / args.steps
        A = csr.to_scipy()
        rel = float(np.linalg.norm(b - A @ x.cpu().numpy()) / np.linalg.norm(b))
        # the split of a step, outside the timed region: the setup alone, then
        # the solve alone, each between synchronisations (medians over the
        # steps, after one untimed split)
        t_setup, t_solve = [], []
        for rep in range(args.steps + 1):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            p_ = pp.setup(M, v0d, d, basis=args.setup_basis if inner == "fp32" else "fp64")
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            pp.solve(p_, M, bd, tol=tol, m=m, inner=inner)
            torch.cuda.synchronize()
            if rep:
                t_setup.append(t2 - t1)
                t_solve.append(time.perf_counter() - t2)
        res[inner] = dict(t=t, info=info, poly=poly, relres=rel, x=x.cpu().numpy(),
                          setup_ms=round(float(np.median(t_setup)) * 1e3, 3),
                          solve_ms=round(float(np.median(t_solve)) * 1e3, 3))
        log(inner, f"time-to-solution {t * 1e3:.1f} ms", info, "true relres", rel,
            f"(split: setup {res[inner]['setup_ms']:.2f} ms, solve {res[inner]['solve_ms']:.2f} ms;",
            "setup runs", [round(v * 1e3, 2) for v in t_setup], "solve runs", [round(v * 1e3, 2) for v in t_solve], ")")

    # p(A)v and phi(A)v bandwidth, FP32 and FP64: the bytes the launches must
    # move by their definition (pp_chain_bytes: format data, vectors,
    # accumulator) over HIP-event time on the stream the library launches on.
    # The CSR-equivalent rate (CSR bytes per product: int32 indices and values) is reported
    # beside it, labelled; it is not a fraction of any kernel's traffic.
    poly = res["fp32"]["poly"]
    pav, phi = {}, {}
    for prec, dt, sv, sx in (("fp32", torch.float32, 4, 4), ("fp64", torch.float64, 8, 8)):
        rp = chain_rate(pp, torch, np, M, poly, prec, dt, args.pav_reps, kind="p")
        nl = poly.d_eff - 1  # sparse products of the p chain
        rp["csr_equiv_GBps"] = (nl * step_bytes(n, nnz, sv, sx) + 2 * n * sx) / (rp["ms"] * 1e-3) / 1e9
        pav[prec] = rp
        log("p(A)v", prec, f"{rp['ms']:.3f} ms", f"{rp['GBps']:.0f} GB/s own bytes", f"{rp['launch_us']:.2f} us/launch")
        # phi(A)v: the Arnoldi operator; d_eff launches of one chain step each
        # unless two steps share a launch
        rf = chain_rate(pp, torch, np, M, poly, prec, dt, args.pav_reps, kind="phi")
        rf["remap"] = M.variant(prec)[1]
        rf["step_us"] = rf["ms"] * 1e3 / poly.d_eff
        rf["csr_step_bytes"] = step_bytes(n, nnz, sv, sx)
        phi[prec] = rf
        log("phi(A)v", prec, f"{rf['ms']:.3f} ms", f"{rf['launch_us']:.2f} us/launch", rf["variant"],
            f"{rf['GBps']:.0f} GB/s own bytes")

    k32 = phi["fp32"]
    for prec in ("fp32", "fp64"):
        if M.march(prec)[0] == 2 and M.march_shape(prec) == 1:
            phi[prec]["variant"] += "/tile2"  # two steps per launch on whole grid lines
    tr = recorded_traffic("fp32", k32["variant"], k32["remap"])
    log("recorded traffic", tr)
    roofline = {
        "bound": "hbm",
        "kernel": chain_kernel_name(k32["variant"]),
        "achieved": round(k32["GBps"], 1),
        "peak": HBM_PEAK_GBPS,
        "unit": "GB/s",
        "frac": round(k32["frac"], 4),
        "traffic": tr["traffic_bytes"] if tr else None,
        "bytes_per_launch": int(round(k32["bytes_per_launch"])),
        "avg_launch_us": round(k32["launch_us"], 3),
        "note": ("achieved = the bytes the FP32 phi(A)v launches must move by their definition (pp_chain_bytes: "
                 "the format's matrix data, one input read, the final vector, one output write) / HIP-event time "
                 "per launch over back-to-back phi(A)v chains on the 3-D 128^3 matrix; traffic = rocprofv3 "
                 "FETCH_SIZE + WRITE_SIZE per launch (copy-calibrated)"),
        "traffic_GBps": round(tr["traffic_bytes"] / (k32["launch_us"] * 1e-6) / 1e9, 1) if tr else None,
        "csr_equiv": {"bytes_per_step": k32["csr_step_bytes"],
                      "GBps": round(k32["csr_step_bytes"] / (k32["step_us"] * 1e-6) / 1e9, 1),
                      "note": "CSR bytes of one product (int32 indices, 4-byte values) over the step time: a "
                              "format-independent work rate, not bytes this kernel moves"},
        "fp64": {"kernel": phi["fp64"]["variant"], "avg_launch_us": round(phi["fp64"]["launch_us"], 3),
                 "bytes_per_launch": int(round(phi["fp64"]["bytes_per_launch"])),
                 "achieved": round(phi["fp64"]["GBps"], 1), "frac": round(phi["fp64"]["frac"], 4)},
    }
    # the kernel boundary: empty launches of the dominant launch's grid
    # (two-step tiles: 16 x 4 lines of the 128 x 128 planes, 1024 threads;
    # one step: 1024 points per workgroup of 256 threads)
    tiles = k32["variant"] == "box/tile2"
    blocks, threads = ((-(-N // 16) * -(-N // 4), 1024) if tiles else (-(-n // 1024), 256))
    floor = launch_floor_us(pp, torch, blocks, threads)
    hbm_us = k32["bytes_per_launch"] / (HBM_PEAK_GBPS * 1e3)
    roofline["launch_floor"] = {
        "blocks": blocks, "threads": threads, "us": round(floor, 3), "hbm_us": round(hbm_us, 3),
        "bound_us": round(floor + hbm_us, 3), "frac_of_bound": round((floor + hbm_us) / k32["launch_us"], 4),
        "note": ("back-to-back empty kernels of the dominant launch's grid (pp_launch_floor, HIP events): the "
                 "cost of a kernel boundary; bound_us = that floor + the launch's bytes at peak HBM bandwidth, a "
                 "lower bound on one launch that the HBM fraction alone does not show at this size")}
    log("launch floor", blocks, "blocks", f"{floor:.2f} us", "bound", f"{floor + hbm_us:.2f} us",
        "achieved", f"{k32['launch_us']:.2f} us")

    extras = {}
    if not args.no_extras:
        extras["random_sparse"] = random_sparse_leg(pp, torch, np)
        extras["chain_step_256"] = scale_leg(pp, torch, np)
        extras["adjoint"] = adjoint_leg(pp, torch, np)
        extras["batched"] = batched_leg(pp, torch, np, orth=args.batch_orth, graph_steps=args.batch_graph_steps)
        extras["preconditioned"] = preconditioned_leg(pp, torch, np)
        extras["paper_context"] = paper_context_leg(pp, torch, np)

    cpu = None
    if not args.no_cpu:
        log("timing the oracle on the host (full time-to-solution)")
        cpu = cpu_baseline(csr, b, v0, d, m, reps=max(1, args.cpu_reps),
                           gpu_x={k: res[k]["x"] for k in ("fp32", "fp64")})

    r32, r64 = res["fp32"], res["fp64"]
    out = {
        "metric": METRIC,
        "value": round(r32["t"], 6),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r32["t"] * 1e3, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"3-D convection-diffusion {N}^3 (n={n}, nnz={nnz}), PP({d}+{poly.n_added})-GMRES({m}) "
                         f"to 1e-8, FP32 chains + FP64 refinement; setup included"),
            "n": n, "nnz": nnz, "d": d, "d_eff": poly.d_eff, "m": m, "tol": tol,
            "setup_basis": args.setup_basis,
        },
        "relres": r32["relres"],
        "x_err_vs_oracle": cpu["x_err_vs_oracle"] if cpu else None,
        "iters": r32["info"]["iters"],
        "cycles": r32["info"]["cycles"],
        "fp64_time_to_solution_s": round(r64["t"], 6),
        "fp64_relres": r64["relres"],
        "fp64_iters": r64["info"]["iters"],
        "mixed_speedup_vs_fp64": round(r64["t"] / r32["t"], 3),
        "split_ms": {"note": "one step split into the setup alone and the solve alone, each between synchronisations, "
                             "measured after the timed steps (medians)",
                     "fp32": {"setup": r32["setup_ms"], "solve": r32["solve_ms"]},
                     "fp64": {"setup": r64["setup_ms"], "solve": r64["solve_ms"]}},
        "pAv_GBps": {"fp32": round(pav["fp32"]["GBps"], 1), "fp64": round(pav["fp64"]["GBps"], 1),
                     "bytes": {"fp32": pav["fp32"]["bytes"], "fp64": pav["fp64"]["bytes"]},
                     "note": "bytes the p(A)v launches must move (pp_chain_bytes) / HIP-event time"},
        "pAv_csr_equiv_GBps": {"fp32": round(pav["fp32"]["csr_equiv_GBps"], 1),
                               "fp64": round(pav["fp64"]["csr_equiv_GBps"], 1)},
        "pAv_ms": {"fp32": round(pav["fp32"]["ms"], 4), "fp64": round(pav["fp64"]["ms"], 4)},
        "matrix_create_s": round(t_create, 6),
        "tune_s": round(t_tune, 6),
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    out.update(extras)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
