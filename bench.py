"""Benchmark: CPR-FGMRES time-to-solution on fully implicit black-oil Jacobians.

One step = the whole hot path for one Newton system of the workload: Jacobian
and right-hand side assembly (bo_jacobian_bsr), CPR setup for that Jacobian
(bo_cpr_update: decoupling, AMG hierarchy and ILU factors rebuilt in the
handle's memory) and the FGMRES(30) solve to a true relative residual of 1e-6
(bo_fgmres_solve).
Steps cycle through the 10 systems of the synthetic step sequence; all inputs
are resident in HBM before timing starts.

Prints one JSON line with the time per system (`value`, seconds), the SpMV
roofline figure (the solver's SpMV launches in the timed steps, timed with HIP
events on the library's stream) and the CPU oracle timed on a bounded sample.
"""
import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "CPR-FGMRES time-to-solution (s) at rel. residual 1e-6; BSR SpMV HBM GB/s"
HBM_PEAK_GBS = 8000.0


# The CPR configuration timed per workload: the library's defaults with the
# smoothing and tile choices measured fastest there (the full-size parity
# tests run the same options on both sides).  Dual porosity (condensed):
# V(3,3) cycles, ILU tiles of 16x4 columns, CPR-FPF; single porosity: V(2,2)
# cycles, 8x8 tiles, two-stage PF.
BENCH_CPR = {"dual": dict(sweeps=3, tile=(16, 4), fpf=1), "grid": dict(sweeps=2, tile=(8, 8), fpf=0)}


def bench_cpr_kw(wl):
    return dict(BENCH_CPR["dual" if wl == 4 else "grid"])


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", type=int, default=4, choices=(0, 1, 2, 4),
                    help="0: 20x20x5; 1: 100x100x50; 2: 200x200x50; 4 (default): dual porosity 400x400x100 "
                         "locations (32M cells) with fixed- BHP and fixed-rate wells")
    ap.add_argument("--systems", type=int, default=0,
                    help="systems of the step sequence to cycle through (default: all 10)")
    ap.add_argument("--form", default="condensed", choices=("condensed", "full"),
                    help="workload 4: 'condensed' (matrix cells eliminated exactly, CPR-FPF on the reduced "
                         "system; default) or 'full' (extended grid form on the whole system)")
    ap.add_argument("--scale", type=int, default=1,
                    help="workload 4 only: divide nx, ny by this (nz by half of it), a smaller twin")
    ap.add_argument("--spmv-isolated", action="store_true",
                    help="also time isolated SpMV launches (after a cache-evicting pass, and back to back)")
    ap.add_argument("--spmv-reps", type=int, default=20)
    ap.add_argument("--ceiling", action="store_true",
                    help="also time plain 1 GiB streams (read-only reduction, copy) as the HBM ceiling")
    ap.add_argument("--precision", default="fp64", choices=("fp64", "fp32", "bf16"),
                    help="inner stages of the preconditioner: FP64, FP32, or FP32 with BF16 ILU factors")
    ap.add_argument("--graph", type=int, default=0, choices=(0, 1),
                    help="1: replay the preconditioner as a HIP graph; 0: launch its kernels directly (default)")
    ap.add_argument("--orth", type=int, default=None, choices=(0, 1, 2),
                    help="Gram-Schmidt form (default: the library's): 0 MGS, 1 CGS2, 2 CGS2 with the "
                         "re-orthogonalisation delayed one step")
    ap.add_argument("--fpf", type=int, default=None, choices=(0, 1),
                    help="CPR form: 1 Algorithm CPR-FPF, 0 two-stage P then F (default: FPF on workload 4, "
                         "two-stage otherwise)")
    ap.add_argument("--model", default="blackoil", choices=("blackoil", "twophase", "pressure"),
                    help="twophase: the oil-water model (2x2 blocks) on workloads 0-2, same grids, rock, "
                         "wells and step sequence without the gas phase; pressure: one scalar pressure "
                         "system, GMRES(30) with RAS-ILU(0) for a fixed 90 iterations (see --pressure-size)")
    ap.add_argument("--pressure-size", default="node", choices=("share", "node"),
                    help="pressure model: 'share' 125x125x47 (3e9 / 4096 unknowns, one process's share of "
                         "the paper's largest run) or 'node' 1000x750x500 (3e9 / 8, one GPU's share on an "
                         "8-GPU node)")
    ap.add_argument("--krylov", default="fgmres", choices=("fgmres", "bicgstab"),
                    help="outer Krylov solver (BiCGSTAB: no per-SpMV timing; use --spmv-isolated)")
    ap.add_argument("--sweeps", type=int, default=None, help="AMG pre- and post-smoothing sweeps (default 1)")
    ap.add_argument("--theta", type=float, default=None, help="AMG strength threshold (default 0.08)")
    ap.add_argument("--tile", type=int, nargs=2, default=None, help="F-stage ILU tile (default 8 8)")
    ap.add_argument("--fstage", default="tiled", choices=("tiled", "natural"),
                    help="F stage: tiled block ILU(0) (default) or block ILU(0) of the whole system in natural "
                         "order by level scheduling (FP64, plain and condensed forms)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quiet", action="store_true")
    return ap.parse_args()


def log(args, *a):
    if not args.quiet:
        print(*a, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU runs are not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.model == "pressure":
        return pressure_main(args)
    import numpy as np
    import torch
    import bo_casegen as cg
    from paper_1606_00556_amd import bo as B

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    wl = args.workload
    twop = args.model == "twophase"
    if twop and wl == 4:
        print(json.dumps({"error": "the two-phase model runs on workloads 0, 1 and 2"}))
        sys.exit(2)
    bs = 2 if twop else 3
    nsys = args.systems or cg.N_SYSTEMS
    systems = [0] if wl == 0 else list(range(1, nsys + 1))
    log(args, f"[bench] generating workload {wl} ({len(systems)} systems)")
    # each system's states go to the device as soon as they are generated
    # (the host keeps the first case's fields for the problem description)
    states = []
    c0 = None
    for k in systems:
        c = cg.make_cfg4(k, scale=args.scale) if wl == 4 else (cg.make_case(wl, k) if wl else cg.make_case(0))
        if twop:
            c = cg.two_phase(c)
            states.append((torch.from_numpy(cg.state2(c.x_old)).to(dev), torch.from_numpy(cg.state2(c.x_new)).to(dev),
                           c.dt))
        else:
            states.append((torch.from_numpy(c.x_old).to(dev), torch.from_numpy(c.x_new).to(dev), c.dt))
        if c0 is None:
            c0 = c
        log(args, f"[bench] generated system {k}: {c.rows} block rows")
    prob = B.problem_from_case(c0, dev)
    n, nnzb = B.bo_jacobian2_bsr_size(prob) if twop else B.bo_jacobian_bsr_size(prob)
    J = (B.DeviceBsr2 if twop else B.DeviceBsr)(torch.empty(n + 1, dtype=torch.int32, device=dev),
                                                torch.empty(nnzb, dtype=torch.int32, device=dev),
                                                torch.empty(bs * bs * nnzb, dtype=torch.float64, device=dev))
    b = torch.empty(bs * n, dtype=torch.float64, device=dev)
    x = torch.empty(bs * n, dtype=torch.float64, device=dev)
    if twop and args.precision != "fp64":
        print(json.dumps({"error": "the two-phase path is FP64 only"}))
        sys.exit(2)
    prec = {"fp64": B.BO_PREC_FP64, "fp32": B.BO_PREC_FP32, "bf16": B.BO_PREC_FP32_BF16}[args.precision]
    condensed = wl == 4 and args.form == "condensed"
    if wl == 4:
        # condensed: every matrix cell eliminated exactly, CPR on the reduced
        # system (fracture cells and fixed-rate wells: pressure system over all
        # of its rows, l1-Jacobi level 0, tiled ILU over the fracture tiles with
        # the wells as a class of their own), Algorithm CPR-FPF.  full: the
        # extended grid form over all 2N cells and the wells, whose mixed forms
        # use block Jacobi.
        grid = (c0.nx, c0.ny, c0.nz, 1)
        # the tiled ILU's FP32 / BF16 factors need a form without matrix cells
        ft = B.BO_F_ILU_TILED if prec == B.BO_PREC_FP64 or condensed else B.BO_F_BJ
        copts = B.bo_cpr_default_opts(precision=prec, ftype=ft, smoother=B.BO_SMOOTH_L1,
                                      npr=0 if condensed else c0.rows, condense=int(condensed))
    else:
        grid = (c0.nx, c0.ny, c0.nz)
        copts = B.bo_cpr_default_opts(precision=prec)
    kw = bench_cpr_kw(wl)
    for k, v in kw.items():
        if k == "tile":
            copts.tile_x, copts.tile_y = v
        else:
            setattr(copts, k, v)
    if args.fpf is not None:
        copts.fpf = args.fpf
    for k, v in (("sweeps", args.sweeps), ("theta", args.theta)):
        if v is not None:
            setattr(copts, k, v)
    if args.tile is not None:
        copts.tile_x, copts.tile_y = args.tile
    if args.fstage == "natural":
        copts.ftype = B.BO_F_ILU_NATURAL
    fo = {"graph": args.graph}
    if args.orth is not None:
        fo["orth"] = args.orth
    fopts = B.bo_fgmres_default_opts(**fo)
    fopts_timed = B.bo_fgmres_default_opts(timing=1, **fo)
    torch.cuda.synchronize()

    # the preconditioner handle lives across systems, as in a Newton loop:
    # bo_cpr_update rebuilds decoupling, AMG hierarchy and ILU factors from
    # scratch for each new Jacobian and only reuses device memory
    assemble = B.bo_jacobian2_bsr if twop else B.bo_jacobian_bsr
    update = B.bo_cpr2_update if twop else B.bo_cpr_update
    solve = {("fgmres", False): B.bo_fgmres_solve, ("bicgstab", False): B.bo_bicgstab_solve,
             ("fgmres", True): B.bo_fgmres_solve2, ("bicgstab", True): B.bo_bicgstab_solve2}[(args.krylov, twop)]
    xo, xn, dt = states[0]
    assemble(prob, xo, xn, dt, J, b)
    pc = B.bo_cpr2_setup(J, grid, copts) if twop else B.bo_cpr_setup(J, grid, copts)

    def step(i, record=None):
        xo, xn, dt = states[i % len(states)]
        e = [torch.cuda.Event(enable_timing=True) for _ in range(4)] if record is not None else None
        if e: e[0].record(stream)
        assemble(prob, xo, xn, dt, J, b)
        if e: e[1].record(stream)
        update(pc, J)
        if e: e[2].record(stream)
        x.zero_()
        info = solve(pc, J, b, x, fopts if record is None else fopts_timed)
        if e: e[3].record(stream)
        if not info["converged"]:
            raise RuntimeError(f"system {i} did not converge: {info}")
        if record is not None:
            record.append((e, info))
        return info

    for w in range(args.warmup):
        info = step(w)
        log(args, f"[bench] warmup {w}: its={info['iterations']} rel={info['rel_residual']:.2e}")
    torch.cuda.synchronize()
    rec = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(args.warmup + k, rec)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = 1000.0 * (t1 - t0) / args.steps
    asm_ms = sum(e[0].elapsed_time(e[1]) for e, _ in rec) / len(rec)
    setup_ms = sum(e[1].elapsed_time(e[2]) for e, _ in rec) / len(rec)
    solve_ms = sum(e[2].elapsed_time(e[3]) for e, _ in rec) / len(rec)
    its = [inf["iterations"] for _, inf in rec]
    log(args, f"[bench] {args.steps} steps: {ms_per_step:.2f} ms/step, assembly {asm_ms:.2f}, setup {setup_ms:.2f}, "
              f"solve {solve_ms:.2f} ms, iterations {its}")

    # SpMV roofline: algorithmic bytes = 72 B per stored block (3x3 FP64) +
    # 24 B x read + 24 B y written per block row (structured indices: the
    # column indices the sliced kernel also reads are not counted), divided by
    # the average duration of the solver's own Arnoldi SpMVs over the timed
    # steps (HIP events recorded by the library on this stream around each
    # launch).  The condensed form's solver multiplies by the reduced system:
    # N fracture rows and the wells, without the 3 blocks per location of the
    # fracture-matrix pairs.
    spmv_calls = sum(inf.get("spmv_calls", 0) for _, inf in rec)
    spmv_us = 1000.0 * sum(inf.get("spmv_ms", 0.0) for _, inf in rec) / max(spmv_calls, 1)
    op_rows = c0.n + c0.nrate if condensed else n
    op_nnzb = nnzb - 3 * c0.n if condensed else nnzb
    spmv_bytes = 8.0 * bs * bs * op_nnzb + 16.0 * bs * op_rows
    spmv_gbs = spmv_bytes / (spmv_us * 1e-6) / 1e9 if spmv_calls else None
    spmv = {"us": spmv_us, "GBs": spmv_gbs, "bytes": spmv_bytes, "launches": spmv_calls}
    if args.spmv_isolated:
        spmv.update(isolated_spmv(args, B, pc, op_rows, dev, stream, bs))
        if spmv_gbs is None:
            spmv_gbs = spmv_bytes / (spmv["isolated_cold_us"] * 1e-6) / 1e9
            spmv["GBs"] = spmv_gbs
    if args.ceiling:
        spmv.update(stream_ceiling(args, dev, stream))
    # plain copy of known size: calibrates the HBM byte counters of a profile
    # taken of this run (FETCH_SIZE / WRITE_SIZE of this copy vs 256 MiB)
    src = torch.ones(1 << 25, dtype=torch.float64, device=dev)
    cal = torch.empty_like(src)
    cal.copy_(src)
    torch.cuda.synchronize()
    del src, cal
    pc.close()
    if spmv_calls:
        log(args, f"[bench] SpMV in the solver: {spmv_us:.1f} us avg over {spmv_calls} launches = "
                  f"{spmv_gbs:.0f} GB/s algorithmic ({spmv_bytes / 1e6:.1f} MB)")

    cpu = None
    if not args.no_cpu_baseline:
        if wl == 4:
            # a bounded sample: the 100x100x50-location twin (1/32 of the
            # cell rows, the same recipe), scaled by the cell ratio and by the
            # iteration ratio (the full-size iterations are the GPU's, which
            # equal the oracle's wherever both were run)
            twin = cg.make_cfg4(systems[0], scale=4)
            cpu = cpu_baseline(args, twin, wl, condensed, twop)
            its_full = sum(its) / len(its)
            f_cells = c0.rows / twin.rows
            f_its = its_full / max(cpu["iterations"], 1)
            cpu["measured_s"] = cpu["value"]
            cpu["value"] = cpu["value"] * f_cells * f_its
            cpu["sample"] = (f"{twin.name} (the same recipe on 100x100x50 locations, {twin.rows} rows): Jacobian "
                             f"+ CPR setup + FGMRES solve by the single-threaded oracle, {cpu['measured_s']:.2f} s "
                             f"for {cpu['iterations']} iterations, scaled x{f_cells:.2f} (rows) "
                             f"x{f_its:.2f} (the GPU's mean {its_full:.1f} iterations at full size)")
        else:
            cpu = cpu_baseline(args, c0, wl, condensed, twop)
    fdesc = ("natural-order BILU0 (level-scheduled)" if args.fstage == "natural"
             else f"tiled BILU0 {copts.tile_x}x{copts.tile_y}")
    out = {
        "metric": METRIC,
        "value": ms_per_step / 1000.0,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f64 (Krylov, residuals) + f32 (AMG, ILU)",
                  "bf16": "f64 (Krylov, residuals) + f32 (AMG) + bf16-stored ILU factors"}[args.precision],
        "data": "synthetic",
        "config": {
            "workload": (f"cfg{wl}: {c0.nx}x{c0.ny}x{c0.nz} "
                         + ("dual-porosity locations with fixed-rate wells, " if wl == 4 else "")
                         + ("two-phase oil-water 2x2-block" if twop else "black-oil 3x3-block")
                         + f" Jacobians ({n} block rows, {bs * n} unknowns, {nnzb} blocks), "
                         + (f"{len(systems)} systems of the synthetic 30-day step sequence" if wl else "one system")),
            "solver": (("BiCGSTAB" if args.krylov == "bicgstab" else "FGMRES(30)")
                       + f", CPR-{'FPF' if copts.fpf else 'PF'}: block quasi-IMPES, SA-AMG V({copts.sweeps},"
                       f"{copts.sweeps}) RB-GS/l1-Jacobi, " + fdesc
                       if wl != 4 else
                       "matrix cells eliminated exactly; FGMRES(30) on the reduced system (fracture cells and "
                       f"fixed-rate wells), CPR-{'FPF' if copts.fpf else 'PF'}: block quasi-IMPES over all of its "
                       f"rows, SA-AMG V({copts.sweeps},{copts.sweeps}) l1-Jacobi, " + fdesc
                       + " (fracture cells, wells); true residual of the full system"
                       if condensed else
                       "FGMRES(30), CPR-FPF extended grid form: block quasi-IMPES over cell and well rows, "
                       f"SA-AMG V({copts.sweeps},{copts.sweeps}) l1-Jacobi, tiled BILU0 {copts.tile_x}x"
                       f"{copts.tile_y} (fracture tiles, matrix cells, wells)"),
            "precision": args.precision,
            "rtol": 1e-6,
            "step": (("bo_jacobian2_bsr + bo_cpr2_update" if twop else "bo_jacobian_bsr + bo_cpr_update")
                     + " (full rebuild, memory reused) + "
                     + {("fgmres", False): "bo_fgmres_solve", ("bicgstab", False): "bo_bicgstab_solve",
                        ("fgmres", True): "bo_fgmres_solve2", ("bicgstab", True): "bo_bicgstab_solve2"}[
                         (args.krylov, twop)]),
            "parallelism": "1 GPU",
        },
        "breakdown_ms": {"assembly": asm_ms, "setup": setup_ms, "solve": solve_ms},
        "iterations": its,
        "spmv": spmv,
        "roofline": {"bound": "hbm", "achieved": spmv_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": spmv_gbs / HBM_PEAK_GBS if spmv_gbs else None,
                     "traffic": None if twop else spmv_traffic(wl, condensed),
                     "traffic_unit": "B per launch",
                     "kernel": "k_slot2_spmv" if twop else ("k_slot_spmv" if wl != 4 else "k_sell_spmv")},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


# HBM traffic summaries of the timed SpMV kernels (rocprofv3 FETCH_SIZE /
# WRITE_SIZE scaled by a 256 MiB copy), per workload: (file, source file,
# kernel, launcher)
TRAFFIC = {
    (1, False): ("slot_spmv_cfg1_500k_hbm_traffic.md", "bo_linalg.hip", "k_slot_spmv(int nx", "bo_status slot_spmv("),
    (4, True): ("sell_spmv_cfg4_condensed_32m_hbm_traffic.md", "bo_linalg.hip", "k_sell_spmv(int n",
                "bo_status sell_spmv("),
}


def kernel_source_hash(src_file, kernel, launcher):
    """sha256 over the text of a kernel and its launcher (the kernel's
    template helpers are not included)."""
    src = open(os.path.join(ROOT, "paper_1606_00556_amd", "csrc", src_file)).read()
    k0 = src.rindex("__global__", 0, src.index(kernel))
    k1 = src.index("\n}\n", k0) + 3
    w0 = src.index(launcher)
    w1 = src.index("\n}\n", w0) + 3
    return hashlib.sha256((src[k0:k1] + src[w0:w1]).encode()).hexdigest()


def spmv_traffic(wl, condensed):
    """HBM bytes per SpMV launch from the committed counter summary, or None
    where there is none or once the kernel source differs from the one the
    counters were taken of."""
    key = (wl, bool(condensed))
    if key not in TRAFFIC:
        return None
    fname, src_file, kernel, launcher = TRAFFIC[key]
    try:
        text = open(os.path.join(ROOT, "profiles", fname)).read()
    except OSError:
        return None
    m_t = re.search(r"traffic per launch \(bytes\): (\d+)", text)
    m_h = re.search(r"kernel source sha256: ([0-9a-f]{64})", text)
    if not (m_t and m_h) or m_h.group(1) != kernel_source_hash(src_file, kernel, launcher):
        return None
    return float(m_t.group(1))


def stream_ceiling(args, dev, stream):
    """The box's streaming ceiling beside the 8 TB/s nominal: a 1 GiB
    read-only reduction and a 1 GiB copy (torch's kernels), each launch after
    a 1 GiB read that evicts L2 and the Infinity Cache, HIP events around the
    launch as for the SpMV."""
    import torch
    nd = 1 << 27
    a = torch.ones(nd, dtype=torch.float64, device=dev)
    c = torch.empty_like(a)
    flush = torch.ones(nd, dtype=torch.float64, device=dev)
    sink = torch.zeros(1, dtype=torch.float64, device=dev)
    out = {}
    for name, op, nbytes in (("read", lambda: torch.sum(a, dim=0, keepdim=True, out=sink), 8.0 * nd),
                             ("copy", lambda: c.copy_(a), 16.0 * nd)):
        for _ in range(2):
            op()
        ev = []
        for _ in range(args.spmv_reps):
            torch.sum(flush, dim=0, keepdim=True, out=sink)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            op()
            e1.record(stream)
            ev.append((e0, e1))
        torch.cuda.synchronize()
        us = 1000.0 * sorted(x.elapsed_time(y) for x, y in ev)[len(ev) // 2]
        out[f"ceiling_{name}_GBs"] = nbytes / (us * 1e-6) / 1e9
        log(args, f"[bench] ceiling {name}: {nbytes / 1e9:.2f} GB in {us:.1f} us (median) = "
                  f"{out[f'ceiling_{name}_GBs']:.0f} GB/s")
    return out


def isolated_spmv(args, B, pc, n, dev, stream, bs=3):
    """SpMV launches outside the solver: each after a 1 GiB read-only pass
    (clean lines, nothing to write back) that evicts L2 and the 256 MB
    Infinity Cache, and back to back (matrix partly cache-resident)."""
    import torch
    xin = torch.randn(bs * n, dtype=torch.float64, device=dev)
    yout = torch.empty_like(xin)
    flush = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    sink = torch.zeros(1, dtype=torch.float64, device=dev)
    for _ in range(3):
        B.bo_cpr_spmv(pc, 1.0, xin, 0.0, yout)
    cold = []
    for _ in range(args.spmv_reps):
        torch.sum(flush, dim=0, keepdim=True, out=sink)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        B.bo_cpr_spmv(pc, 1.0, xin, 0.0, yout)
        e1.record(stream)
        cold.append((e0, e1))
    torch.cuda.synchronize()
    cold_us = 1000.0 * sum(a.elapsed_time(b_) for a, b_ in cold) / len(cold)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record(stream)
    for _ in range(args.spmv_reps):
        B.bo_cpr_spmv(pc, 1.0, xin, 0.0, yout)
    ev[1].record(stream)
    torch.cuda.synchronize()
    warm_us = 1000.0 * ev[0].elapsed_time(ev[1]) / args.spmv_reps
    log(args, f"[bench] isolated SpMV: after eviction {cold_us:.1f} us, back to back {warm_us:.1f} us")
    return {"isolated_cold_us": cold_us, "isolated_back_to_back_us": warm_us}


def cpu_baseline(args, case, wl, condensed, twop=False):
    """The FP64 oracle on the host: one system (assembly + setup + solve) of
    `case` with the benchmark's CPR options."""
    from oracle import oracle as O
    log(args, "[bench] cpu baseline: oracle on one system")
    t0 = time.perf_counter()
    P = O.Problem(case)
    if twop:
        from oracle import twophase as T
        rp, ci, val, R = T.jacobian(O, P)
        x, info = T.fgmres(O, rp, ci, val, -R, T.Cpr2(O, P, rp, ci, val))
        rp = None
    else:
        rp, ci, val, R = O.jacobian(P)
    kw = bench_cpr_kw(wl)
    oft = O.F_ILU_NATURAL if args.fstage == "natural" else O.F_ILU_TILED
    if rp is None:
        pass
    elif wl == 4 and condensed:
        cond = O.Condensed(P, rp, ci, val, ftype=oft, smoother=O.SMOOTH_L1, **kw)
        x, info = O.condensed_fgmres(rp, ci, val, -R, cond)
    elif wl == 4:
        pc = O.Cpr(P, rp, ci, val, ftype=oft, smoother=O.SMOOTH_L1, npr=P.rows, **kw)
        x, info = O.fgmres(rp, ci, val, -R, pc)
    else:
        pc = O.Cpr(P, rp, ci, val, ftype=oft, **kw)
        x, info = O.fgmres(rp, ci, val, -R, pc)
    t1 = time.perf_counter()
    log(args, f"[bench] cpu baseline: {t1 - t0:.2f} s, its={info['iterations']}")
    return {"value": t1 - t0, "unit": "s", "cores": 1, "kind": "oracle",
            "sample": f"{case.name}: one of the workload's systems, Jacobian + CPR setup + FGMRES solve, "
                      f"single-threaded C oracle, {info['iterations']} iterations",
            "iterations": info["iterations"], "host_cpus": os.cpu_count(), "cpu_model": cpu_model()}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def pressure_main(args):
    """One scalar pressure system solved by GMRES(30) with RAS-ILU(0) (6x6
    tiles, overlap 1) for a fixed 90 iterations, as in the paper's
    linear-solver run; a step = RAS setup + the 90-iteration solve."""
    import numpy as np
    import torch
    import bo_casegen as cg
    from paper_1606_00556_amd import bo as B
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    dims = {"share": (125, 125, 47), "node": (1000, 750, 500)}[args.pressure_size]
    log(args, f"[bench] generating the pressure system {dims}")
    c = cg.pressure_case(*dims)
    coef = torch.from_numpy(c.coef.reshape(-1)).to(dev)
    b = torch.from_numpy(c.b).to(dev)
    del c.coef
    x = torch.zeros(c.n, dtype=torch.float64, device=dev)
    fo = B.bo_fgmres_default_opts(flexible=0, maxit=90, rtol=1e-300, timing=1)
    ro = B.bo_ras_default_opts()
    torch.cuda.synchronize()
    log(args, f"[bench] uploaded {c.n} cells")

    # the handle lives across steps (as across the Newton iterations of a
    # run): bo_ras_update refactors in its memory
    pc = B.bo_ras_setup(dims, coef, ro)

    def step(record=None):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record(stream)
        B.bo_ras_update(pc, coef)
        e[1].record(stream)
        x.zero_()
        info = B.bo_scalar_solve(pc, coef, b, x, fo)
        e[2].record(stream)
        torch.cuda.synchronize()
        if info["iterations"] != 90:
            raise RuntimeError(f"expected 90 iterations: {info}")
        if record is not None:
            record.append((e, info))
        return info

    for w in range(args.warmup):
        info = step()
        log(args, f"[bench] warmup {w}: rel residual after 90 its {info['rel_residual']:.3e}")
    rec = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(rec)
    torch.cuda.synchronize()
    ms = 1000.0 * (time.perf_counter() - t0) / args.steps
    setup_ms = sum(e[0].elapsed_time(e[1]) for e, _ in rec) / len(rec)
    solve_ms = sum(e[1].elapsed_time(e[2]) for e, _ in rec) / len(rec)
    calls = sum(inf["spmv_calls"] for _, inf in rec)
    spmv_us = 1000.0 * sum(inf["spmv_ms"] for _, inf in rec) / max(calls, 1)
    spmv_bytes = 72.0 * c.n      # 7 coefficients, x and y, 8 B each, per row
    gbs = spmv_bytes / (spmv_us * 1e-6) / 1e9
    log(args, f"[bench] {args.steps} steps: {ms:.1f} ms/step, setup {setup_ms:.1f}, solve {solve_ms:.1f} ms; "
              f"SpMV {spmv_us:.1f} us = {gbs:.0f} GB/s")
    cpu = None
    if not args.no_cpu_baseline and args.pressure_size == "share":
        from oracle import pressure as PR
        c2 = cg.pressure_case(*dims)
        t = time.perf_counter()
        _, oi = PR.solve(c2, tile=(6, 6), overlap=1, m=30, maxit=90)
        cpu = {"value": time.perf_counter() - t, "unit": "s", "cores": 1, "kind": "oracle",
               "sample": f"the same system, RAS setup + 90 GMRES(30) iterations (C RAS, numpy GMRES)"}
    out = {
        "metric": "GMRES(30)+RAS-ILU(0) time for 90 iterations on one pressure system (s)",
        "value": ms / 1000.0, "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"scalar 7-point pressure system {dims[0]}x{dims[1]}x{dims[2]} ({c.n} unknowns)",
                   "solver": "GMRES(30), right-preconditioned, CGS2 with the second projection delayed one "
                             "step, 90 fixed iterations; RAS 6x6 tiles, overlap 1, ILU(0) subdomain solves",
                   "step": "bo_ras_update (refactor in place) + bo_scalar_solve", "parallelism": "1 GPU"},
        "breakdown_ms": {"setup": setup_ms, "solve": solve_ms},
        "rel_residual_90": rec[-1][1]["rel_residual"],
        "spmv": {"us": spmv_us, "GBs": gbs, "bytes": spmv_bytes, "launches": calls},
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gbs / HBM_PEAK_GBS, "traffic": None, "kernel": "k_scalar_spmv"},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
