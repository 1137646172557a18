"""Training and evaluation driver of the learned pressure-stage correction.

Pairs come from the solver itself (bo_cpr_collect_pairs: the pressure-stage
inputs r_p of a CPR-FGMRES solve and the error e = A_pp^{-1} r_p - V(r_p) the
V-cycle leaves), on seeded training fields of the 200x200x50 workload's recipe
(bo_casegen, cfg 3); the network is trained on the GPU by the library's own
forward, backward and Adam kernels on random crops; evaluation solves the
workload's own systems (cfg 2) with and without the network attached.

Every step of the method runs in the library's kernels; torch holds device
memory, and cropping and batching the pairs is tensor indexing.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field as dfield
from typing import List, Optional

import numpy as np

from . import bo as B


@dataclass
class Pair:
    x: object          # [nz, ny, nx, 2] float32: r_p / s and the standardised ln k
    e: object          # [nz, ny, nx] float32: e / s
    name: str = ""
    coef: object = None  # [7, nz, ny, nx] float32: the pressure stencil, each row scaled by its diagonal


def standardised_logk(case):
    lk = np.log(case.kx)
    return ((lk - lk.mean()) / lk.std()).astype(np.float32)


def _system(case, dev):
    import torch
    p = B.problem_from_case(case, dev)
    J, b = B.bo_jacobian_bsr(p, torch.from_numpy(case.x_old).to(dev), torch.from_numpy(case.x_new).to(dev),
                             case.dt)
    return p, J, b


def collect_pairs(cases, precision=B.BO_PREC_FP32, ncalls=4, rtol_inner=1e-8, log=None) -> List[Pair]:
    """Pairs from the first `ncalls` pressure-stage calls of a CPR-FGMRES
    solve of each case (the plain grid form with the given precision)."""
    import torch
    dev = torch.device("cuda:0")
    pairs = []
    for c in cases:
        _, J, b = _system(c, dev)
        pc = B.bo_cpr_setup(J, (c.nx, c.ny, c.nz), B.bo_cpr_default_opts(precision=precision))
        r, e, got = B.bo_cpr_collect_pairs(pc, b, ncalls=ncalls, rtol_inner=rtol_inner)
        coef = B.bo_cpr_pressure_stencil(pc).reshape(7, c.nz, c.ny, c.nx)
        coef = (coef / coef[3]).contiguous()   # rows scaled by their diagonal (Jacobi): balanced cells
        z = torch.from_numpy(standardised_logk(c)).to(dev).reshape(c.nz, c.ny, c.nx)
        for q in range(got):
            rq = r[q].reshape(c.nz, c.ny, c.nx)
            s = torch.sqrt(torch.mean(rq.double() * rq.double())).float()
            x = torch.stack([rq / s, z], dim=-1).contiguous()
            pairs.append(Pair(x, (e[q].reshape(c.nz, c.ny, c.nx) / s).contiguous(), f"{c.name}#{q}", coef))
        pc.close()
        del J, b
        if log:
            log(f"pairs from {c.name}: {got}")
    return pairs


@dataclass
class TrainLog:
    losses: List[float] = dfield(default_factory=list)
    seconds: float = 0.0
    fwd_ms: float = 0.0
    bwd_ms: float = 0.0
    voxels_per_step: int = 0


def train(nn: B.Nn, pairs: List[Pair], steps=2000, batch=4, crop=(32, 64, 64), lr=1e-3, lr_final=1e-4,
          seed=0, log=None, log_every=250, weighted=False) -> TrainLog:
    """Adam on random crops (batch crops per step, each from a randomly drawn
    pair) of the mean squared error, or (weighted) of the A_pp-weighted error:
    the pressure residual the correction would leave, the judge's measure;
    the learning rate decays geometrically from lr to lr_final."""
    import torch
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(seed)
    cz, cy, cx = crop
    X = torch.empty((batch, cz, cy, cx, 2), dtype=torch.float32, device=dev)
    T = torch.empty((batch, cz, cy, cx), dtype=torch.float32, device=dev)
    K = torch.empty((7, batch, cz, cy, cx), dtype=torch.float32, device=dev) if weighted else None
    out = torch.empty_like(T)
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    tl = TrainLog(voxels_per_step=batch * cz * cy * cx)
    fwd = bwd = 0.0
    nt = 0
    t0 = time.perf_counter()
    for it in range(steps):
        for q in range(batch):
            p = pairs[int(rng.integers(len(pairs)))]
            nz, ny, nx = p.e.shape
            z0, y0, x0 = (int(rng.integers(0, max(nz - cz, 0) + 1)), int(rng.integers(0, max(ny - cy, 0) + 1)),
                          int(rng.integers(0, max(nx - cx, 0) + 1)))
            X[q].copy_(p.x[z0:z0 + cz, y0:y0 + cy, x0:x0 + cx])
            T[q].copy_(p.e[z0:z0 + cz, y0:y0 + cy, x0:x0 + cx])
            if weighted:
                K[:, q].copy_(p.coef[:, z0:z0 + cz, y0:y0 + cy, x0:x0 + cx])
        timed = it % 50 == 10
        if timed:
            ev[0].record(stream)
        nn.forward(X, out)
        if timed:
            ev[1].record(stream)
        loss = nn.backward_weighted(K, T) if weighted else nn.backward(T)
        if timed:
            ev[2].record(stream)
        a = lr * (lr_final / lr) ** (it / max(steps - 1, 1))
        nn.adam_step(a)
        tl.losses.append(loss)
        if timed:
            torch.cuda.synchronize()
            fwd += ev[0].elapsed_time(ev[1])
            bwd += ev[1].elapsed_time(ev[2])
            nt += 1
        if log and (it % log_every == 0 or it == steps - 1):
            log(f"step {it}: loss {loss:.4e} lr {a:.2e}")
    torch.cuda.synchronize()
    tl.seconds = time.perf_counter() - t0
    tl.fwd_ms = fwd / max(nt, 1)
    tl.bwd_ms = bwd / max(nt, 1)
    return tl


# flops of one forward pass per voxel: 2 x 27 taps x sum of c_in c_out
FWD_FLOP_PER_VOXEL = 2 * 27 * sum(a * b for a, b in zip(B.NN_CHANNELS[:-1], B.NN_CHANNELS[1:]))


def evaluate(nn: Optional[B.Nn], cases, precision=B.BO_PREC_FP32, repeats=3, log=None):
    """Solves each case with the plain pressure stage and with the network
    attached (same handle, same options): iterations, kept corrections and
    the median solve time of `repeats` runs (HIP events on the stream)."""
    import torch
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    rows = []
    for c in cases:
        _, J, b = _system(c, dev)
        pc = B.bo_cpr_setup(J, (c.nx, c.ny, c.nz), B.bo_cpr_default_opts(precision=precision))
        logk = torch.from_numpy(np.log(c.kx)).to(dev)
        res = {}
        for attach in ((False, True) if nn is not None else (False,)):
            B.bo_cpr_attach_nn(pc, nn if attach else None, logk if attach else None)
            times = []
            for _ in range(repeats):
                x = torch.zeros_like(b)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                info = B.bo_fgmres_solve(pc, J, b, x)
                e1.record(stream)
                torch.cuda.synchronize()
                times.append(e0.elapsed_time(e1))
            r = b.clone()
            B.bo_bsr_spmv(J, -1.0, x, 1.0, r)
            rel = float(torch.linalg.norm(r) / torch.linalg.norm(b))
            res[attach] = dict(iterations=info["iterations"], used=info["nn_used"], converged=info["converged"],
                               ms=sorted(times)[len(times) // 2], rel=rel)
        rows.append((c.name, res))
        if log:
            msg = f"{c.name}: AMG {res[False]['iterations']} its {res[False]['ms']:.1f} ms"
            if True in res:
                msg += (f"; AMG+network {res[True]['iterations']} its {res[True]['ms']:.1f} ms "
                        f"(corrections kept {res[True]['used']})")
            log(msg)
        B.bo_cpr_attach_nn(pc, None)
        pc.close()
    return rows


def main(argv=None):
    """Pairs from training fields of the 200x200x50 recipe, training, and the
    comparison on the workload's own systems; one JSON line of results."""
    import argparse
    import json
    import sys
    import bo_casegen as cg
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--fields", type=int, default=8, help="training fields (seeds 1606300 + f)")
    ap.add_argument("--systems", default="1,5,9", help="systems of each field's step sequence to collect from")
    ap.add_argument("--steps", type=int, default=3000, help="Adam steps (4 crops of 32x64x64 each)")
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--weighted", action="store_true", help="train on the A_pp-weighted error instead of the MSE")
    ap.add_argument("--eval", default="1,4,7,10", help="systems of the 200x200x50 workload to solve")
    ap.add_argument("--save", default="", help="write the trained parameters here (.npy)")
    a = ap.parse_args(argv)

    def log(*m):
        print(*m, file=sys.stderr, flush=True)

    systems = [int(v) for v in a.systems.split(",")]
    t0 = time.perf_counter()
    pairs = []
    for f in range(a.fields):
        pairs += collect_pairs([cg.make_case(3, k, field=f) for k in systems], log=log)
    t_pairs = time.perf_counter() - t0
    nn = B.Nn(cg.cnn_init(1606300))
    tl = train(nn, pairs, steps=a.steps, lr=a.lr, lr_final=a.lr / 10, weighted=a.weighted, log=log)
    vox = tl.voxels_per_step
    fwd_tf = FWD_FLOP_PER_VOXEL * vox / (tl.fwd_ms * 1e-3) / 1e12
    bwd_tf = 2 * FWD_FLOP_PER_VOXEL * vox / (tl.bwd_ms * 1e-3) / 1e12
    if a.save:
        np.save(a.save, nn.get()[0])
    rows = evaluate(nn, [cg.make_case(2, k) for k in [int(v) for v in a.eval.split(",")]], log=log)
    out = dict(pairs=len(pairs), fields=a.fields, systems=systems, pair_seconds=t_pairs, steps=a.steps,
               loss="weighted" if a.weighted else "mse", loss_first=float(np.mean(tl.losses[:50])),
               loss_last=float(np.mean(tl.losses[-200:])), train_seconds=tl.seconds,
               forward_ms=tl.fwd_ms, backward_ms=tl.bwd_ms, voxels_per_step=vox,
               forward_tflops=fwd_tf, backward_tflops=bwd_tf,
               solves=[dict(system=n, plain=r[False], network=r[True]) for n, r in rows])
    print(json.dumps(out), flush=True)
    return out


if __name__ == "__main__":
    main()
