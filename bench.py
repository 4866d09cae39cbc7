"""Benchmark of the fused collide-and-stream step on one MI355X.

Default workload: the body-force-driven D3Q27 Smagorinsky channel with the
Spalding wall model on both walls, 384 x 192 x 192 cells, FP32 deviation
storage (14.2 M cells, 1.53 GB of populations).  One step = wall prepass +
fused bulk collide-and-stream + wall reconstruction over the whole domain.

Prints one JSON line: MLUPS over all cells (value), the roofline entry of the
dominant kernel (the bulk collide-and-stream kernel, timed with HIP events
recorded on its own stream over the timed steps), the rate of that kernel's
access pattern without the collision (pattern_ceiling), and the FP64 CPU
oracle timed on a bounded crop of the same workload on the host cores.  On
the default channel workload the line also carries the adjoint/forward step
time ratio of the porosity workload and the FP16-storage moment error
against FP32 storage.

Usage: python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline]
Workloads: channel (default), channel16, urban, urban16, big, big16 (1024^3
urban-style domain, the largest that fits one GPU), urban_slip, urban_slip16
(full-slip side and top faces), cavity, cavity16, tgv, adjoint (reverse /
forward step time), precision (FP32 and FP16 storage against FP64 on the
same GPU), cavity_sweep (the cavity at one GPU's share of each problem of
the strong-scaling table, 12 M to 762 M cells), wall_balance (the channel's
mean modeled wall stress against the body force at statistical steady state;
--spinup, --steps, --sample-every).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E peak


def storage_bytes(storage):
    return {"f64": 8, "f32": 4, "f16": 2}[storage]


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("kernels.hip", "lattice.h", "internal.h"):
        with open(os.path.join(ROOT, "paper_2506_21804_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def make_case(name):
    from paper_2506_21804_amd import inputs as I
    if name in ("channel", "channel16"):
        return I.channel(384, 192, 192, q=27), ("f16" if name.endswith("16") else "f32"), \
            "channel384x192x192_d3q27_smag_wallmodel"
    if name in ("urban", "urban16"):
        return I.urban(768, 768, 256, q=27, with_wall_dist=False), ("f16" if name.endswith("16") else "f32"), \
            "urban768x768x256_d3q27_smag_wallmodel_fringe_lid"
    if name in ("urban_open", "urban_open16"):
        return I.urban(768, 768, 256, q=27, with_wall_dist=False, open_x=True), \
            ("f16" if name.endswith("16") else "f32"), "urban768x768x256_d3q27_smag_wallmodel_inlet_outlet_fringe_lid"
    if name in ("urban_slip", "urban_slip16"):
        return I.urban(768, 768, 256, q=27, with_wall_dist=False, slip_walls=True), \
            ("f16" if name.endswith("16") else "f32"), "urban768x768x256_d3q27_smag_wallmodel_fringe_fullslip_sides_top"
    if name in ("big", "big16"):
        case = I.urban(1024, 1024, 1024, q=27, with_wall_dist=False, x_lo=64, x_hi=896, host_fields=False)
        case.u0 = I.urban_u0_device(case)
        return case, ("f16" if name.endswith("16") else "f32"), "urban1024x1024x1024_d3q27_smag_wallmodel_fringe_lid"
    if name == "tgv":
        return I.taylor_green(32, q=19), "f64", "tgv32_d3q19_smag"
    if name in ("cavity", "cavity16"):
        return I.cavity(575, q=19), ("f16" if name.endswith("16") else "f32"), "cavity575_d3q19_smag_lid"
    if name == "adjoint":
        return I.porous_channel(128), "f32", "porous_channel128_d3q19_adjoint"
    raise SystemExit(f"unknown workload {name}")


def measured_traffic(workload, collision, fd_weight, profiles=None):
    """HBM bytes per bulk launch from the committed counter file of this
    workload, or None.  Counter-measured bytes apply only to the kernel they
    were taken on: the same sources, workload, collision and
    finite-difference weight."""
    tf = os.path.join(profiles or os.path.join(ROOT, "profiles"), f"k_bulk_{workload}_traffic.json")
    if not os.path.exists(tf):
        return None
    with open(tf) as fh:
        t = json.load(fh)
    if (t.get("kernel_hash") == kernel_source_hash() and t.get("collision") == collision
            and t.get("fd_weight") == fd_weight):
        return t.get("bytes_per_launch")
    return None


def open_face_cells(case):
    """Fluid cells of the inlet and outlet planes that are not lid cells (the
    open-face kernel updates them, the bulk kernel skips them)."""
    if not case.open_x:
        return 0
    nx, ny, nz = case.shape
    m = np.ones((nz, ny, nx), bool) if case.mask is None else np.asarray(case.mask).reshape(nz, ny, nx) != 0
    if case.lid:
        m = m[:-1]
    return int(m[:, :, 0].sum() + m[:, :, -1].sum())


def cpu_baseline(name, budget_s=12.0, collision=0, fd_weight=0.0):
    """The FP64 oracle on a bounded crop of the workload (same x-y plane,
    fewer z planes), timed around its step loop on the host cores."""
    import oracle as O
    from paper_2506_21804_amd import inputs as I
    if name.startswith("channel"):
        case = I.channel(384, 192, 24, q=27)
        sample = "channel crop 384x192x24 (walls at z), D3Q27 FP64"
    elif name.startswith("urban") or name.startswith("big"):
        open_x = name.startswith("urban_open")
        slip = name.startswith("urban_slip")
        case = I.urban(192, 192, 128, q=27, fringe_len=32, x_lo=16, x_hi=144, h_mean=20.0, h_max=48, open_x=open_x,
                       slip_walls=slip)
        sample = "urban crop 192x192x128 (buildings, fringe, {}{}), D3Q27 FP64".format(
            "full-slip sides and top" if slip else "lid", ", inlet and outlet" if open_x else "")
    elif name == "tgv":
        case = I.taylor_green(32, q=19)
        sample = "tgv 32^3 D3Q19 FP64 (full)"
    elif name.startswith("cavity"):
        case = I.cavity(128, q=19)
        sample = "cavity 128^3 D3Q19 FP64 (same recipe, smaller box)"
    else:
        case = I.porous_channel(shape=(128, 128, 16))
        sample = "porous channel crop 128x128x16 D3Q19 FP64"
    case.collision = collision
    case.fd_weight = fd_weight
    if collision:
        sample += ", recursive regularized collision"
    if fd_weight > 0:
        sample += f", hybrid with finite-difference weight {fd_weight}"
    p = O.make_params(case.q, case.shape, periodic=case.periodic, tau0=case.tau0, cs_smag=case.cs_smag,
                      force=case.force, wall_model=case.wall_model, kappa=case.kappa, E=case.E,
                      fringe_len=case.fringe_len, u_ref=case.u_ref, z0=case.z0, lid=case.lid,
                      collision=case.collision, fd_weight=case.fd_weight, open_x=case.open_x, rho_out=case.rho_out)
    s = O.Oracle(p, mask=case.mask, wall_dist=case.wall_dist, porosity=case.porosity, rho0=case.rho0, u0=case.u0)
    t0 = time.perf_counter()
    s.step(1)
    one = time.perf_counter() - t0
    n = max(1, min(1000, int(budget_s / max(one, 1e-6)) - 1))
    t0 = time.perf_counter()
    s.step(n)
    dt = time.perf_counter() - t0
    cores = O.num_threads()
    # the same crop on one thread, on a quarter of the budget
    O.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        s.step(1)
        one1 = time.perf_counter() - t0
        n1 = max(1, min(1000, int(budget_s / 4 / max(one1, 1e-6))))
        t0 = time.perf_counter()
        s.step(n1)
        dt1 = time.perf_counter() - t0
    finally:
        O.set_num_threads(cores)
    return {"value": round(case.ncells * n / dt / 1e6, 3), "unit": "MLUPS", "cores": cores,
            "kind": "oracle", "sample": f"{sample}, {n} steps, {dt:.1f} s",
            "one_thread": {"value": round(case.ncells * n1 / dt1 / 1e6, 3), "cores": 1,
                           "sample": f"same crop, {n1} steps, {dt1:.1f} s"}}


def calibration_copy(torch, nbytes=4 << 30):
    """One device copy of nbytes (a torch copy_): the known-size kernel the
    FETCH_SIZE / WRITE_SIZE counters are scaled by."""
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    torch.cuda.empty_cache()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="channel")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate", action="store_true",
                    help="also run one 4 GiB device copy (the reference kernel of the PMC traffic calibration)")
    ap.add_argument("--no-ceiling", action="store_true",
                    help="skip the access-pattern ceiling (the bulk kernel's loads and stores without the collision)")
    ap.add_argument("--no-extras", action="store_true",
                    help="channel: skip the adjoint ratio and the FP16-vs-FP32 error added to the line")
    ap.add_argument("--collision", default="bgk", choices=["bgk", "rr3"],
                    help="bulk collision model: BGK or recursive regularized (third order)")
    ap.add_argument("--vortices", type=int, default=0,
                    help="urban_open workloads: seeded vortex-method seed points on the inlet (intensity 0.1, "
                         "size 4 cells); the time of one inlet-field update is reported")
    ap.add_argument("--fd-weight", type=float, default=0.0,
                    help="with --collision rr3: weight 1 - sigma of the finite-difference strain (hybrid)")
    ap.add_argument("--spinup", type=int, default=60000, help="wall_balance workload: steps before sampling")
    ap.add_argument("--sample-every", type=int, default=200, help="wall_balance workload: steps between samples")
    ap.add_argument("--no-spread", action="store_true",
                    help="allocate the workspace and adjoint buffers as one plain allocation each instead of with "
                         "their arrays spread in physical memory (lbm_workspace_alloc / lbm_adjoint_alloc)")
    ap.add_argument("--profile-steps", type=int, default=2000,
                    help="precision workload: second horizon, with mean-profile errors")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2506_21804_amd as lbm

    lbm.load()
    torch.cuda.set_device(0)
    if args.workload == "precision":
        return bench_precision(args, torch, lbm)
    if args.workload == "wall_balance":
        return bench_wall_balance(args, torch, lbm)
    if args.workload == "cavity_sweep":
        return bench_cavity_sweep(args, torch, lbm)
    case, storage, wname = make_case(args.workload)
    if args.collision == "rr3":
        case.collision = 1
        wname += "_rr3"
        if args.fd_weight > 0:
            case.fd_weight = args.fd_weight
            wname += f"_hybrid{args.fd_weight:g}"
    print(f"[bench] workload {wname} storage {storage} cells {case.ncells}", file=sys.stderr, flush=True)
    if args.workload == "adjoint":
        return bench_adjoint(args, torch, lbm, case, storage, wname)

    spread = not args.no_spread
    try:
        lat = lbm.Lattice(case, storage=storage, wall_dist=None if case.wall_dist is None else "case", spread=spread)
    except lbm.LbmError as e:
        if not spread:
            raise
        # too little free device memory for the spread pieces: the plain layout
        print(f"[bench] spread workspace unavailable ({e}); plain allocation", file=sys.stderr, flush=True)
        spread = False
        lat = lbm.Lattice(case, storage=storage, wall_dist=None if case.wall_dist is None else "case")
    N = case.ncells
    nfluid = case.nfluid()
    nwall = lbm.lbm_wall_count(lat.ctx)
    n_open = open_face_cells(case)
    vortex_ms = None
    if args.vortices > 0:
        if not case.open_x:
            raise SystemExit("--vortices needs a workload with open x faces (urban_open, urban_open16)")
        rng = np.random.default_rng(2506 + 7)
        yz = np.stack([rng.uniform(0, case.shape[1], args.vortices), rng.uniform(0, case.shape[2], args.vortices)], 1)
        sign = np.where(rng.uniform(size=args.vortices) < 0.5, -1, 1)
        lat.set_vortices(yz, sign, 0.1, 4.0)
        lat.sync()
        t0 = time.perf_counter()
        for _ in range(10):
            lat.set_vortices(yz, sign, 0.1, 4.0)
        lat.sync()
        vortex_ms = (time.perf_counter() - t0) / 10 * 1e3
        wname += f"_vortices{args.vortices}"
    del case
    torch.cuda.empty_cache()
    stream = lat.stream
    lat.step(args.warmup)
    lat.sync()
    print(f"[bench] warmup {args.warmup} done, wall cells {nwall}", file=sys.stderr, flush=True)

    # timed region: exactly K steps, bracketed by device synchronisation
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    lat.step(args.steps)
    ev1.record(stream)
    lat.sync()
    torch.cuda.synchronize()
    wall_s = time.perf_counter() - t0
    ms_total = ev0.elapsed_time(ev1)
    ms_step = ms_total / args.steps
    mlups = N * args.steps / (ms_total * 1e-3) / 1e6
    print(f"[bench] timed {args.steps} steps: {ms_step:.4f} ms/step, {mlups:.1f} MLUPS (host {wall_s:.3f} s)",
          file=sys.stderr, flush=True)
    # five more timed runs of K/5 steps each, for the spread of the step time
    # (K more steps in all: the urban canopy with BGK, which turns unstable
    # after some 1 800 steps, stays within that)
    reps = []
    kr = max(1, args.steps // 5)
    for _ in range(5):
        ev0.record(stream)
        lat.step(kr)
        ev1.record(stream)
        lat.sync()
        reps.append(ev0.elapsed_time(ev1) / kr)
    print(f"[bench] 5 repeats: median {np.median(reps):.4f} ms/step", file=sys.stderr, flush=True)

    # per-kernel times over the same number of steps, events on the library's stream
    lbm.lbm_profile(lat.ctx, True)
    lat.step(args.steps)
    lbm.lbm_profile(lat.ctx, False)
    kms, kcount = lbm.lbm_profile_read(lat.ctx)
    lat.sync()
    k2_ms = kms[1] / max(kcount[1], 1)
    q = lat.q
    sb = storage_bytes(storage)
    fdw = args.fd_weight if args.collision == "rr3" else 0.0
    # algorithmic bytes of one bulk launch: every cell's flag byte, q loads and
    # q stores for each fluid cell it updates (all fluid cells but the wall
    # cells and the open-face cells); the hybrid collision also reads the velocity field once (four
    # compute-type values per fluid cell), which a pre-pass over the q loads
    # of every fluid cell wrote
    rb = 8 if storage == "f64" else 4
    k2_bytes = N * 1 + (nfluid - nwall - n_open) * 2 * q * sb + (nfluid * 4 * rb if fdw > 0 else 0)
    achieved = k2_bytes / (k2_ms * 1e-3) / 1e9
    step_bytes = nfluid * (2 * q * sb + 1) + (nfluid * (q * sb + 8 * rb) if fdw > 0 else 0)
    traffic = measured_traffic(args.workload, args.collision, fdw)
    diag = lat.diagnostics()
    ceiling = None
    if not args.no_ceiling:
        # the same tiles, order, cells and slots as the bulk kernel, loads and
        # stores only: the rate this access pattern reaches on this part
        pms = lbm.lbm_stream_probe(lat.ctx, 40)
        ceiling = {"gbs": round(k2_bytes / (pms * 1e-3) / 1e9, 1), "ms_per_launch": round(pms, 5),
                   "bulk_fraction_of_ceiling": round(pms / k2_ms, 4)}
    out = {
        "metric": "MLUPS (million lattice-cell updates per second) per GPU",
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f32": "f32 (fp32 deviation storage)", "f16": "f32 compute, f16 deviation storage",
                  "f64": "f64"}[storage],
        "data": "synthetic",
        "config": {"workload": wname, "cells": N, "fluid_cells": nfluid, "wall_cells": nwall, "lattice": f"D3Q{q}",
                   "storage": storage, "collision": args.collision,
                   "fd_weight": fdw, "workspace": "spread" if spread else "plain"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic,
                     "kernel": "k_bulk", "avg_launch_ms": round(k2_ms, 5), "alg_bytes_per_launch": k2_bytes},
        "mflups": round(nfluid * args.steps / (ms_total * 1e-3) / 1e6, 2),
        "repeat_ms_per_step": {"median": round(float(np.median(reps)), 5), "min": round(min(reps), 5),
                               "max": round(max(reps), 5), "repeats": 5, "steps_each": kr},
        "step_alg_gbs": round(step_bytes / (ms_step * 1e-3) / 1e9, 1),
        "kernel_ms_per_step": {"wall_prepass_refwall": round(kms[0] / max(kcount[0], 1), 5),
                               "wall": round(kms[2] / max(kcount[2], 1), 5), "bulk": round(k2_ms, 5)},
        "mass_drift_rel": None,
    }
    if ceiling is not None:
        out["pattern_ceiling"] = ceiling
    if vortex_ms is not None:
        # host-timed: copy of the seed points (after a stream synchronisation) and the field kernel
        out["vortex_field_update_ms"] = round(vortex_ms, 4)
    out["mass"] = float(diag[0])
    del lat
    torch.cuda.empty_cache()
    if args.calibrate:
        calibration_copy(torch)
    if args.workload == "channel" and args.collision == "bgk" and not args.no_extras:
        # the metric's other two parts on the same run: the adjoint/forward
        # step-time ratio on the porosity workload, and the FP16-storage
        # moment error against FP32 storage on this channel
        print("[bench] adjoint/forward ratio (porous channel 128^3, FP32)", file=sys.stderr, flush=True)
        out["adjoint"] = adjoint_ratio(torch, lbm, make_case("adjoint")[0], "f32", 300, 20, spread=spread)
        print("[bench] FP16 vs FP32 storage (channel, 100 steps)", file=sys.stderr, flush=True)
        out["fp16_vs_fp32"] = fp16_vs_fp32(torch, lbm)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args.workload, collision=1 if args.collision == "rr3" else 0,
                                           fd_weight=args.fd_weight if args.collision == "rr3" else 0.0)
    out.pop("mass_drift_rel")
    print(json.dumps(out), flush=True)


def bench_precision(args, torch, lbm):
    """FP32- and FP16-deviation storage against FP64 storage on the same GPU,
    from the same initial state (the FP64 path matches the CPU oracle to
    1e-14).  Pointwise errors of rho and u after 100 steps (max-norms relative
    to the FP64 field's max-norm, and the rms of u), and after
    ``--profile-steps`` steps the same plus the error of the mean streamwise
    velocity profile <u_x>(z) (plane averages over fluid cells, relative to
    the FP64 profile's maximum)."""
    from paper_2506_21804_amd import inputs as I
    horizons = (100, args.profile_steps)
    rows = {}

    def errors(ref, rho, u, mask3):
        out = {"rho": float((rho - ref[0]).abs().max() / ref[0].abs().max()),
               "u": float((u - ref[1]).abs().max() / ref[1].abs().max()),
               "u_rms": float(((u - ref[1]) ** 2).mean().sqrt() / (ref[1] ** 2).mean().sqrt())}
        return out

    def profile(u, mask3, shape):
        nx, ny, nz = shape
        ux = u[0].reshape(nz, ny, nx)
        cnt = mask3.sum(dim=(1, 2)).clamp(min=1)
        return (ux * mask3).sum(dim=(1, 2)) / cnt

    def urban_rr():
        # the urban canopy is not stable with BGK over 2000 steps; the
        # recursive regularized collision is
        c = I.urban(768, 768, 256, q=27, with_wall_dist=False)
        c.collision = 1
        return c

    for wname, make in (("channel384x192x192", lambda: I.channel(384, 192, 192, q=27)),
                        ("urban768x768x256_rr3", urban_rr)):
        case = make()
        nx, ny, nz = case.shape
        mask3 = (torch.ones((nz, ny, nx), dtype=torch.float64, device="cuda") if case.mask is None else
                 torch.as_tensor(case.mask.reshape(nz, ny, nx), device="cuda").to(torch.float64))
        res = {f"{h} steps": {} for h in horizons}
        refs = {}
        for storage in ("f64", "f32", "f16"):
            lat = lbm.Lattice(case, storage=storage, wall_dist=None if case.wall_dist is None else "case")
            done = 0
            try:
                for h in horizons:
                    lat.step(h - done)
                    done = h
                    rho, u = lat.moments()
                    rho, u = rho.double(), u.double()
                    prof = profile(u, mask3, case.shape)
                    key = f"{h} steps"
                    if storage == "f64":
                        refs[h] = (rho, u, prof)
                    else:
                        ref = refs[h]
                        e = errors(ref, rho, u, mask3)
                        e["mean_profile_ux"] = float((prof - ref[2]).abs().max() / ref[2].abs().max())
                        res[key][storage] = e
                    del rho, u
            except RuntimeError as exc:  # a run that stops (e.g. non-finite state) is reported, not hidden
                res.setdefault(f"failed by step {done}", {})[storage] = str(exc)
            print(f"[bench] precision {wname} {storage}: {done} steps done", file=sys.stderr, flush=True)
            del lat
            torch.cuda.empty_cache()
        rows[wname] = res
        del case, refs, mask3
        torch.cuda.empty_cache()
        print(f"[bench] precision {wname}: {res}", file=sys.stderr, flush=True)
    ch = rows["channel384x192x192"].get("100 steps", {}).get("f16", {})
    out = {"metric": "moment error of FP32/FP16 deviation storage vs FP64 storage (same GPU, same steps)",
           "value": ch.get("u"), "unit": "max-norm relative error of u (FP16, channel, 100 steps)",
           "n_gpus": 1, "steps": horizons[-1], "warmup": 0, "ms_per_step": None, "higher_is_better": False,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32 compute", "data": "synthetic",
           "config": {"workload": "channel384x192x192 (BGK) and urban768x768x256 (recursive regularized), D3Q27"},
           "errors": rows}
    print(json.dumps(out), flush=True)


def bench_wall_balance(args, torch, lbm):
    """Momentum balance of the wall-modeled channel at statistical steady
    state: the body force on the fluid, F per unit volume over the half
    height h, is carried by the two walls, so the mean modeled wall stress
    <rho u_tau^2> approaches F h.  Runs --spinup steps, then samples the wall
    records every --sample-every steps for --steps steps; reports the ratio
    <rho u_tau^2> / (F h) over the whole sample and over its two halves."""
    from paper_2506_21804_amd import inputs as I
    case = I.channel(384, 192, 192, q=27)
    F, h = case.force[0], case.extra["h"]
    lat = lbm.Lattice(case, storage="f32")
    nwall = lbm.lbm_wall_count(lat.ctx)
    rec_cells = lbm.lbm_wall_records(lat.ctx)["cells"]
    t0 = time.perf_counter()
    done = 0
    while done < args.spinup:
        k = min(5000, args.spinup - done)
        lat.step(k)
        lat.sync()
        done += k
        print(f"[bench] wall balance spin-up {done}/{args.spinup} steps ({time.perf_counter() - t0:.0f} s)",
              file=sys.stderr, flush=True)
    samples, mom = [], [float(lat.diagnostics()[1])]
    for s in range(0, args.steps, args.sample_every):
        lat.step(args.sample_every)
        mom.append(float(lat.diagnostics()[1]))
        rho, _ = lat.moments()
        r = lbm.lbm_wall_records(lat.ctx)
        rw = rho.double().reshape(-1)[torch.as_tensor(rec_cells.astype(np.int64), device="cuda")].cpu().numpy()
        samples.append(float((rw * r["utau"] ** 2).mean()))
        if (s // args.sample_every) % 20 == 0:
            print(f"[bench] wall balance sample {len(samples)}: <rho u_tau^2>/(F h) = {samples[-1] / (F * h):.4f} "
                  f"({time.perf_counter() - t0:.0f} s)", file=sys.stderr, flush=True)
    sm = np.array(samples) / (F * h)
    half = len(sm) // 2
    # the momentum the walls actually take out: each step the forcing adds F
    # per fluid cell to sum c f, so the walls remove F V - dP/dt; over the
    # nwall wall cells this is a mean wall stress to compare with F h
    V = case.ncells if case.mask is None else int(np.count_nonzero(case.mask))
    P = np.array(mom)

    def budget(a, b):
        return (F * V - (P[b] - P[a]) / ((b - a) * args.sample_every)) / (nwall * F * h)
    out = {"metric": "wall-law momentum balance <rho u_tau^2> / (F h) at statistical steady state",
           "value": round(float(sm.mean()), 4), "unit": "ratio", "n_gpus": 1, "steps": args.steps,
           "warmup": args.spinup, "ms_per_step": None, "higher_is_better": None, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32 (fp32 deviation storage)", "data": "synthetic",
           "config": {"workload": "channel384x192x192_d3q27_smag_wallmodel", "wall_cells": nwall,
                      "sample_every": args.sample_every},
           "halves": [round(float(sm[:half].mean()), 4), round(float(sm[half:].mean()), 4)],
           "removed_by_walls": round(float(budget(0, len(sm))), 4),
           "removed_by_walls_halves": [round(float(budget(0, half)), 4), round(float(budget(half, len(sm))), 4)],
           "mean_velocity": [round(float(P[0] / V), 6), round(float(P[-1] / V), 6)],
           "min": round(float(sm.min()), 4), "max": round(float(sm.max()), 4), "samples": len(sm),
           "mass": float(lat.diagnostics()[0])}
    print(json.dumps(out), flush=True)


def bench_cavity_sweep(args, torch, lbm):
    """The lid-driven cavity (D3Q19, FP32 storage, BGK, C_S = 0.1) at one
    GPU's share of each problem of the paper's strong-scaling table (Sec. 3.1:
    575^3 to 1449^3 on 4 to 16 GPUs), taken as an n x n x ceil(n/G) slab of
    the cube: 12 M to 762 M cells per GPU.  Each shape runs on its own as a
    closed box (walls on all faces, lid on top; the halo exchange of a
    multi-GPU run is not part of it) for about half a second of steps.
    Reports MLUPS and the bulk kernel's fraction of the HBM peak per shape;
    value is the median MLUPS over the shapes."""
    from paper_2506_21804_amd import inputs as I
    import numpy as np
    rows = []
    for n in (575, 725, 913, 1150, 1449):
        for G in (4, 8, 16):
            shape = (n, n, -(-n // G))
            case = I.cavity(shape, q=19)
            N = case.ncells
            t0 = time.perf_counter()
            lat = lbm.Lattice(case, storage="f32", spread=not args.no_spread)
            t_init = time.perf_counter() - t0
            steps = int(min(300, max(20, round(0.5 / (N / 3.0e10)))))
            lat.step(10)
            lat.sync()
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ev0.record(lat.stream)
            lat.step(steps)
            ev1.record(lat.stream)
            lat.sync()
            ms = ev0.elapsed_time(ev1) / steps
            lbm.lbm_profile(lat.ctx, True)
            lat.step(10)
            lbm.lbm_profile(lat.ctx, False)
            kms, kcount = lbm.lbm_profile_read(lat.ctx)
            lat.sync()
            k2_ms = kms[1] / max(kcount[1], 1)
            k2_bytes = N * 1 + N * 2 * 19 * 4
            frac = k2_bytes / (k2_ms * 1e-3) / 1e9 / PEAK_HBM_GBS
            finite = bool(np.isfinite(lat.diagnostics()[0]))
            del lat
            torch.cuda.empty_cache()
            rows.append({"cube": n, "gpus": G, "shape": list(shape), "cells": N, "steps": steps,
                         "ms_per_step": round(ms, 4), "mlups": round(N / (ms * 1e-3) / 1e6, 1),
                         "bulk_hbm_frac": round(frac, 4), "finite": finite})
            print(f"[bench] cavity {n}^3 / {G}: {shape} {N / 1e6:.1f} M cells, {ms:.3f} ms/step, "
                  f"{rows[-1]['mlups']:.0f} MLUPS, bulk {frac:.3f} of peak (init {t_init:.1f} s)",
                  file=sys.stderr, flush=True)
    m = [r["mlups"] for r in rows]
    out = {"metric": "MLUPS (million lattice-cell updates per second) per GPU", "value": round(float(np.median(m)), 1),
           "unit": "MLUPS", "n_gpus": 1, "steps": None, "warmup": 10, "ms_per_step": None, "higher_is_better": True,
           "scaling": "strong", "vs_baseline": None, "dtype": "f32 (fp32 deviation storage)", "data": "synthetic",
           "config": {"workload": "cavity_strong_scaling_shares_d3q19_smag_lid", "lattice": "D3Q19",
                      "storage": "f32", "collision": "bgk", "workspace": "plain" if args.no_spread else "spread"},
           "min": min(m), "max": max(m), "shapes": rows}
    print(json.dumps(out), flush=True)


def bench_adjoint(args, torch, lbm, case, storage, wname):
    """Forward step vs hand-written reverse step on the porosity workload,
    and one full checkpointed gradient."""
    r = adjoint_ratio(torch, lbm, case, storage, args.steps, args.warmup, spread=not args.no_spread)
    if args.calibrate:
        calibration_copy(torch)
    out = {
        "metric": "adjoint/forward step time ratio",
        "value": r["ratio"],
        "unit": "ratio",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": r["forward_ms_per_step"],
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": wname, "cells": case.ncells},
    }
    out.update({k: v for k, v in r.items() if k != "ratio"})
    print(json.dumps(out), flush=True)


def adjoint_ratio(torch, lbm, case, storage, K, warmup, spread=True):
    """Median of 5 repeats of K forward steps and of K reverse steps (half at
    each parity) on the porosity workload, their ratio, and one full
    checkpointed gradient (terminal and time-averaged objective, T = 400,
    20 snapshots)."""
    lat = lbm.Lattice(case, storage=storage, spread=spread)
    N = case.ncells
    planes = case.extra["planes"]
    lat.step(warmup)
    lat.sync()
    stream = lat.stream
    e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    torch.cuda.synchronize()
    fwd, adj = [], []
    lam = lat.new_adjoint(spread=spread)
    grad = lat.new_gradient()
    for _ in range(5):
        e[0].record(stream)
        lat.step(K)
        e[1].record(stream)
        lat.sync()
        fwd.append(e[0].elapsed_time(e[1]) / K)
        lbm.lbm_adjoint_seed(lat.ctx, planes, lam)
        lat.sync()
        # half of the reverse steps at each parity (a forward step in between
        # flips the parity; it is outside the timed brackets)
        adj_total = 0.0
        for half in (K // 2, K - K // 2):
            e[2].record(stream)
            for _ in range(half):
                lbm.lbm_adjoint_step(lat.ctx, lam, grad)
            e[3].record(stream)
            lat.sync()
            adj_total += e[2].elapsed_time(e[3])
            lat.step(1)
        adj.append(adj_total / K)
    fwd_ms = float(np.median(fwd))
    adj_ms = float(np.median(adj))
    T, nsnap = 400, 20
    snaps = torch.empty(nsnap * lbm.lbm_state_bytes(lat.ctx), dtype=torch.uint8, device="cuda")
    t0 = time.perf_counter()
    J, nfwd = lbm.lbm_gradient(lat.ctx, T, planes, snaps, nsnap, lam, grad)
    grad_s = time.perf_counter() - t0
    # the time-averaged objective: the same sweep, with the objective taken at
    # every step of the first descent and its seeds fused into the adjoint
    t0 = time.perf_counter()
    Jm, nfwd_m = lbm.lbm_gradient_mean(lat.ctx, T, planes, snaps, nsnap, lam, grad)
    grad_mean_s = time.perf_counter() - t0
    out = {
        "ratio": round(adj_ms / fwd_ms, 3),
        "workload": "porous_channel128_d3q19_adjoint",
        "storage": storage,
        "buffers": "spread" if spread else "plain",
        "forward_ms_per_step": round(fwd_ms, 5),
        "forward_mlups": round(N / (fwd_ms * 1e-3) / 1e6, 1),
        "adjoint_ms_per_step": round(adj_ms, 5),
        "repeats": 5,
        "gradient": {"T": T, "snapshots": nsnap, "forward_steps": nfwd, "seconds": round(grad_s, 3),
                     "J": J, "forward_only_seconds": round(T * fwd_ms * 1e-3, 3)},
        "gradient_time_averaged": {"T": T, "snapshots": nsnap, "forward_steps": nfwd_m,
                                   "seconds": round(grad_mean_s, 3), "J": Jm},
    }
    del lat, lam, grad, snaps
    torch.cuda.empty_cache()
    return out


def fp16_vs_fp32(torch, lbm, steps=100):
    """FP16- against FP32-deviation storage on the channel workload, from the
    same initial state, after ``steps`` steps: max-norm errors of rho and u
    relative to the FP32 field's max-norm, the rms error of u, and the error
    of the mean streamwise profile <u_x>(z)."""
    from paper_2506_21804_amd import inputs as I
    case = I.channel(384, 192, 192, q=27)
    nx, ny, nz = case.shape
    res = {}
    for storage in ("f32", "f16"):
        lat = lbm.Lattice(case, storage=storage)
        lat.step(steps)
        rho, u = lat.moments()
        res[storage] = (rho.double(), u.double())
        del lat
        torch.cuda.empty_cache()
    (r32, u32), (r16, u16) = res["f32"], res["f16"]
    p32 = u32[0].reshape(nz, ny * nx).mean(dim=1)
    p16 = u16[0].reshape(nz, ny * nx).mean(dim=1)
    out = {"workload": "channel384x192x192_d3q27_smag_wallmodel", "steps": steps,
           "rho": float((r16 - r32).abs().max() / r32.abs().max()),
           "u": float((u16 - u32).abs().max() / u32.abs().max()),
           "u_rms": float(((u16 - u32) ** 2).mean().sqrt() / (u32 ** 2).mean().sqrt()),
           "mean_profile_ux": float((p16 - p32).abs().max() / p32.abs().max())}
    del res, r32, u32, r16, u16
    torch.cuda.empty_cache()
    return out


if __name__ == "__main__":
    main()
