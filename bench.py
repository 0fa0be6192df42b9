#!/usr/bin/env python3
"""Throughput of the vectorial lattice Boltzmann hot path on one MI355X.

Headline workload: 2D shallow-water radial dam break, D2Q4 per component
(12 distributions per node), 4096 x 4096 periodic grid, lambda = 6, s = 1.8,
FP64 storage (the paper's arithmetic precision).  One "step" = one pull-stream +
collide pass over the whole grid; the library advances several steps per kernel
launch (temporal blocking, bitwise identical to single steps), so the launch
reads the state once and writes it once for all of them.  `value` is MLUPS
(million lattice-node updates per second) with the state resident in HBM.

Beside it on the same JSON line:
  forms.fp32     the same workload with FP32 storage (FP64 arithmetic), with the L1
                 error of h against the FP64-storage run of the same steps
  forms.*_faces  the same grid with inflow / Neumann / wall faces
  forms.*_one_step_per_launch  the same with one step per launch
  forms.wall_1d_*  1D wall reflection, 2^20 nodes (MALL-resident)
  forms.dam_break_1d  the 1D dam break as stated (1000 nodes, 400 steps, FP64): the
                 whole run's time, set by launch latency
  forms.batched  256 mixed 1D / 2D Riemann problems, FP32 storage, 1000 steps, in
                 the tuned mode (the fused tiles of K steps over every instance in
                 ONE persistent launch for the run, replayed from a captured graph);
                 beside it the other forms (the same tiles as two launches per K
                 steps, the persistent dataflow and step-synchronous modes), the
                 FP64 reference of the FP32 L1 error, the committed DRAM counters of
                 the batched kernels and the plain path launched per instance
  forms.rest_mrt_*  the paper's rest-population schemes with one relaxation rate per
                 non-conserved moment: D2Q5Q4Q4 on the headline grid (FP64 and FP32
                 storage, several steps per launch, the FP32 L1 error of h; FP64 one
                 step per launch beside it), D1Q3Q2 on the 1D wall reflection (16
                 steps per launch; one step beside it) and on the Sec. 2 setup
  forms.entropy_2d_f64  the discrete entropy diagnostic of the headline state
  forms.adjoint  2D 1024^2 gradient rollout (T = 500, checkpoints every 23 steps)
  roofline       the dominant kernel (the FP64 launches of the timed region's most
                 frequent steps per launch) against its binding roof -- FP64 VALU issue or HBM, named
                 from committed rocprofv3 counters -- with both roofs' figures
  cpu_baseline   the CPU FP64 oracle on bounded samples of every workload, at one
                 host thread and at all threads it is given

Usage: python bench.py [--gpus 1] [--steps 2000] [--warmup 20] [--quick]
"""
import argparse
import json
import os
import sys
import time

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s


def _parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=4096, help="grid side of the headline workload")
    ap.add_argument("--quick", action="store_true", help="headline only (no batched/adjoint/cpu)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-1d", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-rest", action="store_true",
                    help="skip the rest-population (MRT) and entropy forms")
    ap.add_argument("--no-faces", action="store_true",
                    help="skip the forward run with inflow / Neumann / wall faces")
    ap.add_argument("--batched-steps", type=int, default=1000,
                    help="timed steps of the batched form (the manifest's run is 1000)")
    ap.add_argument("--batched-tuned-only", action="store_true",
                    help="batched form: the tuned mode only (no FP64 reference, persistent "
                         "modes or per-instance plain path)")
    ap.add_argument("--batch-mode", type=int, default=-1, choices=(-1, 0, 1, 2, 3, 4),
                    help="batched form: mode to time instead of the tuned one (-1)")
    ap.add_argument("--direct-batch", action="store_true",
                    help="batched form: launch every kernel directly instead of replaying "
                         "captured graphs (for profilers)")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--npt", type=int, default=0)
    ap.add_argument("--pad", type=int, default=-1)
    ap.add_argument("--fuse", type=int, default=0, choices=tuple(range(0, 9)),
                    help="steps per launch of the forward form (0 = tuned / library default)")
    ap.add_argument("--probe-copy", action="store_true",
                    help="first run a plain device copy of 2^30 bytes (reference for counters)")
    ap.add_argument("--storage", choices=("both", "f64", "f32"), default="both")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Faces of the bounded forward run: the oblique shock's set (inflow left and top,
# outflow right, wall bottom) around the radial dam break.
FACES = ("inflow", "neumann", "wall", "inflow")
FACES_INFLOW = {0: (1.0, 0.2, 0.0), 3: (1.0, 0.0, -0.2)}


def time_forward(torch, n, storage, steps, warmup, block, npt, pad, fuse=1, keep_h=False,
                 bc=("periodic",) * 4, inflow=None):
    """Forward steps of the headline workload; ``fuse`` = steps per launch asked
    for (0 = the library's choice; lbm_launch_info reports what runs).  The timed
    region issues the library's own plan for ``steps`` steps (lbm_launch_plan:
    launches of K steps, a remainder of two or more spread evenly over the last
    launches) one launch per lbm_step call, with a HIP event on the launch stream
    after each, so the average duration of the launches of the dominant kernel
    (the most frequent steps per launch of the plan) is measured directly.  With
    ``keep_h`` the final height field is returned under "h"."""
    from paper_1401_0427_amd import workloads as W
    from paper_1401_0427_amd.lbm import Solver

    c = W.radial_dam_break_2d(n, lam=6.0)
    S = Solver(2, n, n, lam=c.lam, s=c.s, h0=c.h0, qx0=c.qx0, qy0=c.qy0, storage=storage,
               block=block, npt=npt, plane_pad=pad, fuse_steps=fuse, bc=bc, inflow=inflow)
    info = S.launch_info()
    K = info["steps_per_launch"]
    S.step(warmup)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    pieces = S.launch_plan(steps)
    # the dominant kernel: the most frequent launch depth (ties: the deeper one)
    Kd = max(set(pieces), key=lambda k: (pieces.count(k), k))
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(len(pieces) + 1)]
    t0 = time.perf_counter()
    ev[0].record(st)
    for i, k in enumerate(pieces):
        S.step(k)
        ev[i + 1].record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev[0].elapsed_time(ev[-1])
    dur = [ev[i].elapsed_time(ev[i + 1]) for i in range(len(pieces))]
    full = [d for d, k in zip(dur, pieces) if k == Kd]
    (h, _, _), tot = S.moments(totals=True)
    ok = bool(torch.isfinite(h).all().item()) and tot[0] > 0
    nodes = n * n
    bpl = 12 * 2 * (8 if storage == "f64" else 4)  # algorithmic bytes per lattice update
    out_h = {"h": h.clone()} if keep_h else {}
    # algorithmic bytes of one launch: the state read once and written once, whatever
    # the number of steps the launch advances
    return dict(ms_per_step=ms / steps, mlups=nodes * steps / (ms * 1e-3) / 1e6,
                **out_h, steps_per_launch=K, launches=len(pieces),
                launch_steps={str(k): pieces.count(k) for k in sorted(set(pieces), reverse=True)},
                dominant_steps=Kd, periodic=all(b == "periodic" for b in bc),
                segment_rows=info["segment_rows"], resident_blocks=info["resident_blocks"],
                ms_per_launch=(sum(full) / len(full)) if full else ms / len(pieces),
                full_launches=len(full),
                gbs=nodes * bpl * len(pieces) / (ms * 1e-3) / 1e9, bytes_per_lu=bpl,
                bytes_per_launch=nodes * bpl, wall_s=wall, finite=ok, mass=tot[0])


def time_1d(torch, storage, steps=2000, warmup=64, fuse=0):
    """1D wall reflection, 2^20 nodes (inflow ghost left, wall right, lambda = 3,
    s = 1.9): the state (32 MiB FP64 per buffer) stays in the 256 MB MALL, so the
    rate is reported as effective bandwidth, not as an HBM claim.  ``fuse`` =
    steps per launch (0 = library default)."""
    from paper_1401_0427_amd import workloads as W
    from paper_1401_0427_amd.lbm import Solver

    c = W.wall_reflection_1d()
    S = Solver(1, c.nx, 1, lam=c.lam, s=c.s, bc=c.bc, inflow=c.inflow, h0=c.h0, qx0=c.qx0,
               storage=storage, fuse_steps=fuse)
    S.step(warmup)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    S.step(steps)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    h = S.moments()[0]
    ok = bool(torch.isfinite(h).all().item())
    bpl = 4 * 2 * (8 if storage == "f64" else 4)
    return dict(nodes=c.nx, steps=steps, ms_per_step=ms / steps,
                mlups=c.nx * steps / (ms * 1e-3) / 1e6, effective_gbs=c.nx * bpl * steps / (ms * 1e-3) / 1e9,
                bytes_per_lu=bpl, finite=ok, h=h.clone())


def time_dam_break_1d(torch, reps=20):
    """The 1D dam break as stated (1000 nodes, 400 steps, FP64, Neumann ends), the
    whole run timed from its initial state ``reps`` times: far too small to fill a GPU
    (one workgroup per launch), so launch latency sets the rate."""
    from paper_1401_0427_amd import workloads as W
    from paper_1401_0427_amd.lbm import Solver

    c = W.dam_break_1d()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    S = Solver(1, c.nx, 1, lam=c.lam, s=c.s, bc=c.bc, h0=c.h0, qx0=c.qx0, storage="f64")
    init = S.current()[0].clone()
    S.step(c.steps)  # untimed: first launches
    best = None
    for _ in range(reps):
        S.import_(init)
        torch.cuda.synchronize()
        e0.record(st)
        S.step(c.steps)
        e1.record(st)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    return dict(nodes=c.nx, steps=c.steps, ms_run=best, ms_per_step=best / c.steps,
                mlups=c.nx * c.steps / (best * 1e-3) / 1e6,
                launches=len(S.launch_plan(c.steps)))


# Rest weight and moment rates of the timed rest-population runs (one rate per
# non-conserved moment, Sec. 2 / Sec. 3): 2D (J_x, J_y, eps, XX_rho, f_xx, f_xy, XX_u,
# f_yx, f_yy, XX_v), 1D (J_rho, eps_rho, J_q).
REST_A = 0.05
REST_RATES_2D = (1.7, 1.6, 1.2, 1.9, 1.5, 1.3, 1.1, 1.45, 1.55, 1.8)
REST_RATES_1D = (1.7, 1.3, 1.9)


def time_rest_2d(torch, n, storage, steps=200, warmup=10, fuse=0):
    """D2Q5Q4Q4 with moment-space MRT (the rest-population scheme of Sec. 3) on the
    headline radial dam break: 13 planes, 208 B (FP64) / 104 B (FP32) of state read
    and written per launch and node.  ``fuse`` = steps per launch asked for (0 = the
    library's choice: 5 on this grid; 1 = the one-step kernel, an HBM stream).  Each
    launch of the library's plan is timed with HIP events on the launch stream."""
    from paper_1401_0427_amd import workloads as W
    from paper_1401_0427_amd.lbm import Solver

    c = W.radial_dam_break_2d(n, lam=6.0)
    S = Solver(2, n, n, lam=c.lam, s=c.s, h0=c.h0, qx0=c.qx0, qy0=c.qy0, storage=storage,
               rest=True, a=REST_A, rates=list(REST_RATES_2D), fuse_steps=fuse)
    K = S.launch_info()["steps_per_launch"]
    S.step(warmup)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    pieces = S.launch_plan(steps)
    Kd = max(set(pieces), key=lambda k: (pieces.count(k), k))
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(len(pieces) + 1)]
    ev[0].record(st)
    for i, k in enumerate(pieces):
        S.step(k)
        ev[i + 1].record(st)
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[-1])
    full = [ev[i].elapsed_time(ev[i + 1]) for i, k in enumerate(pieces) if k == Kd]
    (h, _, _), tot = S.moments(totals=True)
    torch.cuda.synchronize()
    hc = h.cpu()
    # the copy's sum against the library's FP64 total of the same moments call
    copy_ok = abs(float(hc.sum()) - tot[0]) <= 1e-9 * abs(tot[0])
    bpl = 13 * 2 * (8 if storage == "f64" else 4)
    ms_launch = sum(full) / len(full)
    gbs = n * n * bpl / (ms_launch * 1e-3) / 1e9
    return dict(ms_per_step=ms / steps, mlups=n * n * steps / (ms * 1e-3) / 1e6,
                steps_per_launch=K, dominant_steps=Kd,
                launch_steps={str(k): pieces.count(k) for k in sorted(set(pieces), reverse=True)},
                ms_per_launch=ms_launch, bytes_per_launch=n * n * bpl, gbs=gbs,
                hbm_frac=gbs / HBM_PEAK_GBS, a=REST_A, rates=list(REST_RATES_2D),
                finite=bool(torch.isfinite(hc).all().item()), mass=tot[0], h=hc,
                h_copy_consistent=copy_ok)


def time_rest_1d(torch, storage="f64", steps=2000, warmup=64, fuse=0):
    """D1Q3Q2 with moment-space MRT (Sec. 2) on the 1D wall reflection (2^20 nodes):
    5 planes, 80 B (FP64) of state per node update; 40 MiB per buffer, so it runs out
    of the MALL and the rate is an effective bandwidth.  ``fuse`` = steps per launch
    (0 = library default, 16 here)."""
    from paper_1401_0427_amd import workloads as W
    from paper_1401_0427_amd.lbm import Solver

    c = W.wall_reflection_1d()
    S = Solver(1, c.nx, 1, lam=c.lam, s=c.s, bc=c.bc, inflow=c.inflow, h0=c.h0, qx0=c.qx0,
               storage=storage, rest=True, a=0.1, rates=list(REST_RATES_1D), fuse_steps=fuse)
    K = S.launch_info()["steps_per_launch"]
    S.step(warmup)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    S.step(steps)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    h = S.moments()[0]
    bpl = 5 * 2 * (8 if storage == "f64" else 4)
    return dict(nodes=c.nx, steps=steps, steps_per_launch=K, ms_per_step=ms / steps,
                mlups=c.nx * steps / (ms * 1e-3) / 1e6,
                effective_gbs=c.nx * bpl * steps / (ms * 1e-3) / 1e9, bytes_per_lu=bpl,
                a=0.1, rates=list(REST_RATES_1D), finite=bool(torch.isfinite(h).all().item()))


def time_fig1_rest_1d(torch, reps=20):
    """The Sec. 2 experiment with the rest population: D1Q3Q2, 80 points, a = 0.15,
    lambda = 8, s = 1.8 on every moment, Neumann ends, 96 steps (the end time is not
    stated; 96 steps of dt = dx / lambda reach t = 0.15), FP64; the whole run timed
    from its initial state ``reps`` times (one launch: the domain fits one tile)."""
    import numpy as np
    from paper_1401_0427_amd import workloads as W
    from paper_1401_0427_amd.lbm import Solver

    n, steps = 80, 96
    x = W.cell_centres(n)
    S = Solver(1, n, 1, lam=8.0, s=1.8, bc=("neumann", "neumann", "periodic", "periodic"),
               h0=np.where(x < 0.5, 2.0, 0.5), qx0=np.zeros(n), storage="f64", rest=True,
               a=0.15, rates=[1.8, 1.8, 1.8])
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    init = S.current()[0].clone()
    S.step(steps)  # untimed: first launches
    best = None
    for _ in range(reps):
        S.import_(init)
        torch.cuda.synchronize()
        e0.record(st)
        S.step(steps)
        e1.record(st)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    return dict(nodes=n, steps=steps, ms_run=best, ms_per_step=best / steps,
                mlups=n * steps / (best * 1e-3) / 1e6, launches=len(S.launch_plan(steps)))


def time_entropy_2d(torch, n, calls=20):
    """The discrete entropy diagnostic (Sec. 1) of the headline state after 16 steps,
    FP64: one pass over the 12 planes (96 B per node) with per-node entropies written
    (8 B per node) and per-block partial sums, then the FP64 totals; each call ends with
    the host reading the totals, so a call is a kernel, a small sum and a copy."""
    from paper_1401_0427_amd import workloads as W
    from paper_1401_0427_amd.lbm import Solver

    c = W.radial_dam_break_2d(n, lam=6.0)
    S = Solver(2, n, n, lam=c.lam, s=c.s, h0=c.h0, qx0=c.qx0, qy0=c.qy0, storage="f64")
    S.step(16)
    H0, bad0 = S.entropy()
    torch.cuda.synchronize()
    best = None
    for _ in range(calls):
        t0 = time.perf_counter()
        H, bad, hn = S.entropy(per_node=True)
        dt = time.perf_counter() - t0
        best = dt if best is None else min(best, dt)
    byt = n * n * (96 + 8)
    return dict(ms_per_call=best * 1e3, bytes_per_call=byt, gbs=byt / best / 1e9,
                hbm_frac=byt / best / 1e9 / HBM_PEAK_GBS, total=H, invalid=bad,
                equals_without_per_node=bool(H == H0 and bad == bad0))


def _manifest_instances():
    from paper_1401_0427_amd import workloads as W

    insts = []
    for m in W.batched_manifest(0):
        h, qx, qy = m.initial()
        bc = ("neumann", "neumann", "periodic", "periodic") if m.dim == 1 else ("periodic",) * 4
        insts.append(dict(dim=m.dim, nx=m.nx, ny=m.ny, lam=m.lam, s=m.s, g=W.G, bc=bc, h0=h,
                          qx0=qx, qy0=qy))
    return insts


def _time_batch(torch, insts, storage, steps, tune):
    """One batch of the manifest: warm-up (graph capture), then `steps` timed with
    HIP events on the launch stream.  Returns (ms, tiles, grid, final packed h)."""
    from paper_1401_0427_amd.lbm import Batch

    B = Batch(insts, storage=storage, **tune)
    B.run(64, check_done=True)  # warm-up; captures the graphs of the chunked modes
    B.run(steps, check_done=True)  # same length as the timed run (persistent modes capture here)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    B.run(steps)
    e1.record(st)
    torch.cuda.synchronize()
    B.check()
    ms = e0.elapsed_time(e1)
    nt, grid = B.info()
    h = B.moments()[0].clone()
    nodes = B.nodes
    del B
    torch.cuda.empty_cache()
    return ms, nt, grid, h, nodes


def time_batched(torch, steps=1000, tuned_only=False, direct=False, mode=-1):
    """The 256-instance manifest (FP32 storage): the tuned mode (the fused tiles of K
    steps over every instance, in one persistent launch for the whole run with a
    grid-wide close per K-step pass, or two launches per K steps), the other modes
    beside it (the persistent dataflow and step-synchronous modes, and the fused
    mode's other form), the same manifest with FP64 storage (the reference of the
    FP32 L1 error, same steps and mode), and the plain path per instance."""
    from paper_1401_0427_amd.lbm import Solver

    insts = _manifest_instances()
    tune = {}
    tpath = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1401_0427_amd",
                         "tuning.json")
    if os.path.exists(tpath):
        tune = json.load(open(tpath)).get("batch", {})
    if mode >= 0 and mode != tune.get("mode"):
        tune = {"mode": mode, "block": 512 if mode == 0 else 256, "tile_nodes": 32768,
                "fuse_steps": tune.get("fuse_steps", 0) if mode >= 3 else 0}
    if direct:
        tune = dict(tune, direct=1)
    ms, nt, grid, h32, nodes = _time_batch(torch, insts, "f32", steps, tune)
    ok = bool(torch.isfinite(h32).all().item())
    byt = sum((4 if i["dim"] == 1 else 12) * 2 * 4 * i["nx"] * (i["ny"] if i["dim"] == 2 else 1)
              for i in insts)
    # algorithmic bytes per launch (persistent fused mode: per pass): each reads and
    # writes every instance's state once, whatever the number of steps it advances
    k = (tune.get("fuse_steps") or 8) if tune.get("mode") in (3, 4) else 1
    out = dict(instances=len(insts), nodes=nodes, steps=steps, ms=ms, ms_per_step=ms / steps,
               mlups=nodes * steps / (ms * 1e-3) / 1e6, steps_per_launch=k,
               gbs=byt * steps / k / (ms * 1e-3) / 1e9, tiles=nt, grid=grid, tuning=tune,
               finite=ok, traffic=_batch_traffic())
    if tuned_only:
        return out
    log("[bench] batched FP64 reference (same mode and steps)")
    _, _, _, h64, _ = _time_batch(torch, insts, "f64", steps, tune)
    out["l1_rel_h_vs_fp64"] = float((h32 - h64).abs().sum() / h64.abs().sum())
    out["l1_ok"] = out["l1_rel_h_vs_fp64"] <= 1e-5
    del h64
    # the persistent forms (every step of every instance in ONE kernel launch) not
    # tuned, and the fused tiles' other form
    fk = tune.get("fuse_steps") or 8
    others = [("dataflow", dict(mode=0, block=512, tile_nodes=32768, pass_nodes=1)),
              ("step_synchronous", dict(mode=1, block=256))]
    if tune.get("mode") == 4:
        others.append(("fused_launch_pairs", dict(mode=3, fuse_steps=fk)))
    else:
        others.append(("fused_passes", dict(mode=4, fuse_steps=fk)))
    pers = {}
    for name, t in others:
        log(f"[bench] batched persistent {name}")
        pms, pnt, pgrid, ph, _ = _time_batch(torch, insts, "f32", steps, t)
        pers[name] = dict(ms_per_step=pms / steps, mlups=nodes * steps / (pms * 1e-3) / 1e6,
                          units=pnt, grid=pgrid, tuning=t,
                          equals_fused=bool(torch.equal(ph, h32)))
    out["persistent"] = pers
    # the plain path, one instance after another (graph-chunked lbm_step), same steps
    psteps = 100
    solvers = [Solver(d["dim"], d["nx"], d["ny"], lam=d["lam"], s=d["s"], bc=d["bc"], h0=d["h0"],
                      qx0=d["qx0"], qy0=d["qy0"] if d["dim"] == 2 else None, storage="f32")
               for d in insts]
    for S in solvers:
        S.step(2)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for S in solvers:
        S.step(psteps)
    e1.record(st)
    torch.cuda.synchronize()
    pms = e0.elapsed_time(e1)
    out["plain_per_instance_mlups"] = nodes * psteps / (pms * 1e-3) / 1e6
    out["speedup_vs_plain"] = out["mlups"] / out["plain_per_instance_mlups"]
    return out


def time_adjoint(torch, n=1024, T=500, K=23, storage="f32"):
    """The adjoint workload: 1024^2, T = 500, FP32 forward, checkpoints every K = 23
    steps.  Timed: the forward rollout and the backward sweep (the backward
    recomputes each segment: one library call per segment), with the adjoint stored
    like the state (the default) and in FP64; beside it the form that keeps every
    level (K = 1: the 501 levels take 24 GB, and one library call runs the whole
    backward sweep with no recomputation), when they fit; the gradients against
    those of the FP64 forward (which equals the CPU FP64 oracle's to 1e-15 in the
    tests); and the adjoint kernel alone against the forward kernel, at 1024^2 and
    at 4096^2 (both HBM-bound)."""
    from paper_1401_0427_amd import workloads as W
    from paper_1401_0427_amd.adjoint import rollout

    c, ht0 = W.adjoint_case(n=n, steps=T)
    target = rollout(torch.as_tensor(ht0, device="cuda"), torch.tensor(c.s, dtype=torch.float64),
                     T, K, lam=c.lam, storage="f64").detach()

    def run(st, adj, k=None):
        h0 = torch.tensor(c.h0, dtype=torch.float64, device="cuda", requires_grad=True)
        s = torch.tensor(c.s, dtype=torch.float64, device="cuda", requires_grad=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hT = rollout(h0, s, T, k, lam=c.lam, storage=st, adjoint_storage=adj)
        loss = ((hT - target) ** 2).sum()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        return t1 - t0, t2 - t1, h0.grad.detach(), float(s.grad)

    from paper_1401_0427_amd.adjoint import every_level_fits

    run(storage, None, K)  # untimed: one-time set-up (module loading, first allocations)
    fwd_s, bwd_s, gh, gs = run(storage, None, K)
    _, bwd64, gh64, gs64 = run(storage, "f64", K)
    _, _, gh_ref, gs_ref = run("f64", None, K)
    every = None
    if every_level_fits(c.h0.shape, T, storage):
        run(storage, None, 1)  # untimed: first allocation of the levels
        fwd_1, bwd_1, gh_1, gs_1 = run(storage, None, 1)
        every = dict(K=1, forward_s=fwd_1, backward_s=bwd_1,
                     grad_mlups=n * n * T / (fwd_1 + bwd_1) / 1e6,
                     same_gradients=bool(torch.equal(gh, gh_1)) and gs == gs_1)

    def rel(a, b):
        return float((a - b).abs().max() / b.abs().max())

    out = dict(n=n, T=T, K=K, storage=storage, adjoint_storage=storage, forward_s=fwd_s,
               backward_s=bwd_s, grad_mlups=n * n * T / (fwd_s + bwd_s) / 1e6,
               every_level=every,
               grad_h0_rel_vs_fp64=rel(gh, gh_ref), grad_s_rel_vs_fp64=abs(gs - gs_ref) / abs(gs_ref),
               backward_s_adjoint_f64=bwd64, grad_h0_rel_vs_fp64_adjoint_f64=rel(gh64, gh_ref),
               grad_s_rel_vs_fp64_adjoint_f64=abs(gs64 - gs_ref) / abs(gs_ref),
               grad_s=gs, grad_h0_norm=float(gh.norm()))
    # adjoint kernel alone: T adjoint steps on resident buffers, FP32 state, FP64
    # and FP32 adjoint, against the forward kernel
    from paper_1401_0427_amd.lbm import Solver

    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    es = 4 if storage == "f32" else 8
    for nb, tb, tag in ((n, T, ""), (4096, 50, "_4096")):
        cb, _ = W.adjoint_case(n=nb, steps=tb)
        for adj in ("f64", "f32"):
            S = Solver(2, nb, nb, lam=cb.lam, s=cb.s, h0=cb.h0, storage=storage, fuse_steps=1,
                       adjoint_storage=adj)
            a, b, u = S.new_adjoint(), S.new_adjoint(), S.current()[0]
            part = S.adjoint_partials()
            S.adjoint_step(u, a, b, part)
            torch.cuda.synchronize()
            e0.record(st)
            for _ in range(tb):
                S.adjoint_step(u, a, b, part)
                a, b = b, a
            e1.record(st)
            torch.cuda.synchronize()
            adj_ms = e0.elapsed_time(e1) / tb
            ea = 4 if adj == "f32" else 8
            out[f"adjoint_step_ms{tag}_adjoint_{adj}"] = adj_ms
            out[f"adjoint_gbs{tag}_adjoint_{adj}"] = nb * nb * 12 * (es + 2 * ea) / (adj_ms * 1e-3) / 1e9
            if adj == "f64":
                e0.record(st)
                S.step(tb)
                e1.record(st)
                torch.cuda.synchronize()
                fwd_ms = e0.elapsed_time(e1) / tb
                out[f"forward_one_step_ms{tag}"] = fwd_ms
                out[f"forward_gbs{tag}"] = nb * nb * 24 * es / (fwd_ms * 1e-3) / 1e9
            del S, a, b, u, part
        torch.cuda.empty_cache()
    out["adjoint_over_forward"] = out["adjoint_step_ms_adjoint_f64"] / out["forward_one_step_ms"]
    out["adjoint_over_forward_4096"] = (out["adjoint_step_ms_4096_adjoint_f64"]
                                        / out["forward_one_step_ms_4096"])
    return out


# FP64 step kernels: (source files, committed traffic summary, committed SQ summary, name)
KERNELS = {
    "one_step": (("fwd.hip", "lbm_device.h"), "k_step2d_fwd_4096_traffic.json",
                 "k_step2d_fwd_4096_sq.json",
                 "k_step2d<double> (fused pull-stream + BGK collide)"),
    "lds_two_step": (("tblock.hip", "lbm_device.h"), "k_step2d_x2_fwd_4096_traffic.json",
                     "k_step2d_x2_fwd_4096_sq.json",
                     "k_step2d_x2<double> (two pull-stream + BGK collide steps per launch)"),
    "wave_strip": (("tblock.hip", "xk_wave.h", "lbm_device.h"), "k_step2d_xk_fwd_4096_traffic.json",
                   "k_step2d_xk_fwd_4096_sq.json",
                   "k_step2d_xk<double, {K}> ({K} pull-stream + BGK collide steps per launch, "
                   "one wavefront per column strip)"),
}

# FP64 operations of one node update as the scheme states them (Sec. 1-3 at a = 0,
# BGK): 2D -- moments 9 additions; equilibria 31 (one division 1/h, p = (g/2) h^2,
# the three fluxes, the scaled flux terms and 12 additions); relaxation
# f + s (f^eq - f) 36.  1D -- 2 + 14 + 12.  A fused multiply-add would count 2.
ALG_FLOPS_2D = 76
ALG_FLOPS_1D = 28
FP64_VECTOR_PEAK_TFLOPS = 78.6  # MI355X: 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz


def kernel_kind(form):
    """Which FP64 step kernel ran the dominant launches of a timed forward form:
    one step per launch, the LDS two-step kernel (two-step launches on
    all-periodic grids), else the wave-strip K-step kernel."""
    if form["dominant_steps"] == 1:
        return "one_step"
    if form["dominant_steps"] == 2 and form["periodic"]:
        return "lds_two_step"
    return "wave_strip"


def _summary(kind, which, n, K):
    """A committed rocprofv3 summary (JSON) of the step kernel (both storages) -- ``which`` 1
    = traffic, 2 = SQ instruction counters -- if it was taken for this grid,
    launch depth and the current kernel source; else None."""
    prof = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles")
    name = KERNELS[kind][which]
    # the summary of the library's default depth, else one taken at K steps per
    # launch (the same name with _k<K> before the counter kind)
    stem, tail = name.rsplit("_", 1)
    for cand in (name, f"{stem}_k{K}_{tail}"):
        path = os.path.join(prof, cand)
        if not os.path.exists(path):
            continue
        d = json.load(open(path))
        if (d.get("n") == n and d.get("kernel_source_sha") == _kernel_sha(kind)
                and d.get("steps_per_launch", K) == K):
            return d
    return None


def _measured_traffic(n, kind, K, storage="f64"):
    """HBM bytes per launch of the step kernel of the given storage (FETCH_SIZE +
    WRITE_SIZE, each scaled by what the counter reads for a plain copy of known
    size)."""
    d = _summary(kind, 1, n, K)
    if d is None:
        return None
    if storage == "f64":
        return d.get("traffic_bytes_per_launch_f64")
    e = d.get(storage)
    return None if e is None else e["read_bytes"] + e["write_bytes"]


def roofline(form, n, kind, storage="f64"):
    """Roofline object of the dominant kernel (the launches of the timed region's
    most frequent depth K, in the storage that was timed).  Both roofs are computed
    from the live launch time; the bound named is the one the kernel uses more of:
    the FP64 VALU issue (busy fraction from the committed SQ counter summary; FP32
    storage computes in FP64 too) or HBM (DRAM bytes from the committed traffic
    summary, else the algorithmic bytes)."""
    K = form["dominant_steps"]
    ms_launch = form["ms_per_launch"]
    nodes = n * n
    alg_bytes = nodes * form["bytes_per_lu"]
    hbm_gbs = alg_bytes / (ms_launch * 1e-3) / 1e9
    tflops = ALG_FLOPS_2D * nodes * K / (ms_launch * 1e-3) / 1e12
    traffic = _measured_traffic(n, kind, K, storage)
    sq = _summary(kind, 2, n, K)
    valu_busy = sq[storage]["valu_busy"] if sq and storage in sq else None
    dram_frac = (traffic if traffic else alg_bytes) / (ms_launch * 1e-3) / 1e9 / HBM_PEAK_GBS
    if valu_busy is not None:
        bound = "alu" if valu_busy > dram_frac else "hbm"
    else:
        bound = "alu" if kind == "wave_strip" else "hbm"
    hbm = {"achieved": round(hbm_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(hbm_gbs / HBM_PEAK_GBS, 4)}
    alu = {"achieved": round(tflops, 3), "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
           "frac": round(tflops / FP64_VECTOR_PEAK_TFLOPS, 4),
           "flops_per_update": ALG_FLOPS_2D}
    main = alu if bound == "alu" else hbm
    return {"bound": bound, "achieved": main["achieved"], "peak": main["peak"],
            "unit": main["unit"], "frac": main["frac"], "traffic": traffic,
            "kernel": KERNELS[kind][3].format(K=K).replace(
                "<double", "<double" if storage == "f64" else "<float"), "steps_per_launch": K,
            "launches_timed": form["full_launches"], "ms_per_launch": round(ms_launch, 5),
            "bytes_per_launch": alg_bytes, "hbm": hbm, "alu": alu,
            "valu_busy": valu_busy, "dram_frac": round(dram_frac, 4),
            "per_step_equivalent_gbs": round(hbm_gbs * K, 1)}


def _sources_sha(files):
    import hashlib

    root = os.path.dirname(os.path.abspath(__file__))
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(root, "paper_1401_0427_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def _kernel_sha(kind="one_step"):
    return _sources_sha(KERNELS[kind][0])


# Sources of the batched kernels (fused, flat and persistent fused modes).
BATCH_SOURCES = ("batch.hip", "pbatch.hip", "tblock.hip", "xk_wave.h", "internal.h",
                 "lbm_device.h")


def _batch_traffic():
    """Committed DRAM counter summary of the batched kernels on the manifest (bytes
    per launch, per pass for the persistent kernel), if taken on the current
    sources; else None."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                        "k_batch_manifest256_traffic.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("kernel_source_sha") != _sources_sha(BATCH_SOURCES):
        return None
    per = {k: {"read_bytes": v["read_bytes"], "write_bytes": v["write_bytes"],
               "over_compulsory": round((v["read_bytes"] + v["write_bytes"]) /
                                        v["algorithmic_bytes"], 4), "per": v.get("per")}
           for k, v in d["kernels"].items()}
    return {"compulsory_bytes_per_pass": d["compulsory_bytes_per_pass"], "kernels": per}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(n):
    """The CPU FP64 oracle as it stands, on bounded samples of every workload, at
    one host thread and at all the threads it is given (OpenMP over nodes; its
    results do not depend on the thread count).  Only the stepping is timed (the
    initial state is built first).  MLUPS = nodes x steps / s; the gradient rate
    is nodes x T / s of the forward + backward sweep, as on the GPU.  The
    headline value is the all-thread rate on the headline workload."""
    import oracle
    from paper_1401_0427_amd import workloads as W

    all_threads = oracle.get_threads()

    def adv(P, f, k):
        import ctypes

        import numpy as np

        g = np.array(f, dtype=np.float64, order="C", copy=True).reshape(-1)
        ptr = g.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        t = time.perf_counter()
        rc = oracle.lib().orc_advance(ctypes.byref(P), ptr, int(k))
        dt = time.perf_counter() - t
        assert rc == 0
        return dt

    runs = {}

    def add(name, sample, nodes_steps, timer):
        row = {"sample": sample}
        for label, th in (("one_thread", 1), ("all_threads", all_threads)):
            oracle.set_threads(th)
            dt = timer(th)
            row[label + "_mlups"] = round(nodes_steps(th) / dt / 1e6, 3)
        oracle.set_threads(all_threads)
        runs[name] = row

    c0 = W.dam_break_1d()
    P0 = oracle.params(1, c0.nx, lam=c0.lam, s=c0.s, g=c0.g, bc=c0.bc)
    f0 = oracle.run(P0, c0.h0, c0.qx0, None, 0)
    add("R0_dam_break_1d", f"{c0.nx} nodes x {c0.steps} steps (the whole run)",
        lambda th: c0.nx * c0.steps, lambda th: adv(P0, f0, c0.steps))
    c1 = W.wall_reflection_1d()
    P1 = oracle.params(1, c1.nx, lam=c1.lam, s=c1.s, g=c1.g, bc=c1.bc, inflow=c1.inflow)
    f1 = oracle.run(P1, c1.h0, c1.qx0, None, 0)
    add("R1_wall_reflection_1d", f"{c1.nx} nodes x 40 steps (of 20000)",
        lambda th: c1.nx * 40, lambda th: adv(P1, f1, 40))
    del f1
    c2 = W.radial_dam_break_2d(n, lam=6.0)
    P2 = oracle.params(2, n, n, lam=c2.lam, s=c2.s, g=c2.g)
    f2 = oracle.run(P2, c2.h0, c2.qx0, c2.qy0, 0)
    k2 = {1: 2}
    add("R2_radial_dam_break_2d", f"{n}x{n} nodes x 2 steps at one thread, 8 at all (of 2000)",
        lambda th: n * n * k2.get(th, 8), lambda th: adv(P2, f2, k2.get(th, 8)))
    del f2
    man = _manifest_instances()
    states = []
    for d in man:
        P = oracle.params(d["dim"], d["nx"], d["ny"], lam=d["lam"], s=d["s"], g=d["g"],
                          bc=d["bc"])
        states.append((P, oracle.run(P, d["h0"], d["qx0"], d["qy0"] if d["dim"] == 2 else None,
                                     0)))
    mnodes = sum(d["nx"] * d["ny"] for d in man)
    add("R3_batched_manifest", f"all {len(man)} instances ({mnodes} nodes) x 1 step (of 1000), "
        "one instance after another",
        lambda th: mnodes, lambda th: sum(adv(P, f, 1) for P, f in states))
    del states
    ca, ht0 = W.adjoint_case(n=1024, steps=500)
    Pa = oracle.params(2, 1024, 1024, lam=ca.lam, s=ca.s, g=ca.g)
    Ta, Ka = 12, 4

    def grad(th):
        t = time.perf_counter()
        oracle.loss_grad_2d(Pa, ca.h0, ht0, Ta, Ka)
        return time.perf_counter() - t

    add("R4_adjoint_gradient_2d", f"1024x1024 nodes, T = {Ta} (of 500), checkpoints every {Ka}: "
        "forward, recompute and adjoint sweep",
        lambda th: 1024 * 1024 * Ta, grad)
    head = runs["R2_radial_dam_break_2d"]
    return {"value": head["all_threads_mlups"], "unit": "MLUPS", "cores": all_threads,
            "kind": "oracle",
            "sample": f"radial dam break {n}x{n}, 8 steps, FP64 C oracle (OpenMP over nodes, "
                      f"{all_threads} threads); other workloads and one thread under 'runs'",
            "cpu_model": _cpu_model(), "runs": runs}


def main():
    args = _parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU sharding is a design "
                                   "note, not implemented", "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    tpath = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1401_0427_amd",
                         "tuning.json")
    fwd_tune = json.load(open(tpath)).get("forward", {}) if os.path.exists(tpath) else {}

    def launch(storage):
        t = fwd_tune.get(storage, {})
        return (args.block or t.get("block", 256), args.npt or t.get("npt", 1),
                args.pad if args.pad >= 0 else t.get("plane_pad", -1),
                args.fuse or t.get("fuse_steps", 0))

    n = args.n
    if args.probe_copy:
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")  # 2^30 bytes
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        log("[bench] copy probe: 2^30 bytes read, 2^30 bytes written")
    forms = {}
    for storage in ("f64", "f32"):
        if args.storage not in ("both", storage):
            continue
        L = launch(storage)
        log(f"[bench] forward {storage.upper()} {n}^2, {args.steps} steps, launch {L}")
        forms["fp" + storage[1:]] = time_forward(torch, n, storage, args.steps, args.warmup, *L,
                                                 keep_h=True)
        if forms["fp" + storage[1:]]["steps_per_launch"] != 1 and not args.quick:
            # the one-step-per-launch kernel on the same workload, for comparison
            log(f"[bench] forward {storage.upper()} {n}^2, one step per launch")
            forms["fp" + storage[1:] + "_one_step_per_launch"] = time_forward(
                torch, n, storage, args.steps, args.warmup, *L[:3], 1)
        if not args.quick and not args.no_faces:
            # the same grid with inflow / Neumann / wall faces (library default launch)
            log(f"[bench] forward {storage.upper()} {n}^2, faces {FACES}")
            forms["fp" + storage[1:] + "_faces"] = time_forward(
                torch, n, storage, args.steps, args.warmup, *L[:3], 0, bc=FACES,
                inflow=FACES_INFLOW, keep_h=True)
    if not args.quick and not args.no_1d:
        for storage in ("f64", "f32"):
            log(f"[bench] 1D wall reflection 2^20 {storage.upper()}")
            forms["wall_1d_" + storage] = time_1d(torch, storage)
        log("[bench] 1D dam break 1000 nodes x 400 steps")
        forms["dam_break_1d"] = time_dam_break_1d(torch)
    # FP32 storage against FP64 storage after the same steps of the same form (the
    # FP64 path equals the CPU FP64 oracle to <= 1e-12 in the parity tests): L1
    # relative error of h, bounded by 1e-5
    for a, b in (("fp32", "fp64"), ("fp32_faces", "fp64_faces"), ("wall_1d_f32", "wall_1d_f64")):
        if a in forms and b in forms:
            h64, h32 = forms[b]["h"], forms[a]["h"]
            e = float((h32 - h64).abs().sum() / h64.abs().sum())
            forms[a]["l1_rel_h_vs_fp64"] = e
            forms[a]["l1_ok"] = e <= 1e-5
    for f in forms.values():
        f.pop("h", None)
    # the headline form: FP64 storage, else (``--storage f32``) FP32 storage
    head_storage = "f64" if "fp64" in forms else "f32"
    f64 = forms["fp" + head_storage[1:]]
    if not args.quick and not args.no_batched:
        log("[bench] batched 256 instances x 1000 steps")
        forms["batched"] = time_batched(torch, steps=args.batched_steps,
                                        tuned_only=args.batched_tuned_only,
                                        direct=args.direct_batch, mode=args.batch_mode)
    if not args.quick and not args.no_rest:
        for storage in ("f64", "f32"):
            log(f"[bench] rest-population MRT 2D {n}^2 {storage.upper()}")
            forms["rest_mrt_2d_" + storage] = time_rest_2d(torch, n, storage)
        log(f"[bench] rest-population MRT 2D {n}^2 F64, one step per launch")
        forms["rest_mrt_2d_f64_one_step_per_launch"] = time_rest_2d(torch, n, "f64", fuse=1)
        forms["rest_mrt_2d_f64_one_step_per_launch"].pop("h")
        # host copies of h taken at the end of each run, each checked against the
        # library's total of the same moments call
        h64, h32 = forms["rest_mrt_2d_f64"].pop("h"), forms["rest_mrt_2d_f32"].pop("h")
        if (forms["rest_mrt_2d_f64"]["h_copy_consistent"]
                and forms["rest_mrt_2d_f32"]["h_copy_consistent"]):
            e = float((h32 - h64).abs().sum() / h64.abs().sum())
            forms["rest_mrt_2d_f32"]["l1_rel_h_vs_fp64"] = e
            forms["rest_mrt_2d_f32"]["l1_ok"] = e <= 1e-5
        else:
            forms["rest_mrt_2d_f32"]["l1_rel_h_vs_fp64"] = None
            forms["rest_mrt_2d_f32"]["l1_ok"] = None
        log("[bench] rest-population MRT 1D 2^20 FP64")
        forms["rest_mrt_1d_f64"] = time_rest_1d(torch)
        log("[bench] rest-population MRT 1D 2^20 FP64, one step per launch")
        forms["rest_mrt_1d_f64_one_step_per_launch"] = time_rest_1d(torch, fuse=1)
        log("[bench] D1Q3Q2 Sec. 2 setup (80 points, 96 steps)")
        forms["rest_mrt_fig1_1d"] = time_fig1_rest_1d(torch)
        log(f"[bench] entropy diagnostic {n}^2 FP64")
        forms["entropy_2d_f64"] = time_entropy_2d(torch, n)
    if not args.quick and not args.no_adjoint:
        log("[bench] adjoint rollout 1024^2 x 500")
        forms["adjoint"] = time_adjoint(torch)
    kind = kernel_kind(f64)
    roof = roofline(f64, n, kind, head_storage)
    cpu = None
    if not args.quick and not args.no_cpu:
        log("[bench] CPU oracle baseline")
        cpu = cpu_baseline(n)
    out = {
        "metric": "MLUPS + % HBM roofline, fwd vs batched vs adjoint, 2D SW 4096² FP64/FP32",
        "value": round(f64["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(f64["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"2D shallow-water radial dam break, D2Q4 x3, {n}x{n} periodic, "
                               f"lambda=6, s=1.8, {head_storage.upper()} storage",
                   "nodes": n * n, "parallelism": "single GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "forms": forms,
        "kernel_source_sha": _kernel_sha(kind),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
