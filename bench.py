#!/usr/bin/env python3
"""Throughput of the MD hot path on one MI355X: atom-steps/s of velocity Verlet
(forces + device-decided neighbour rebuilds + integration + energy sums) on the
1,048,576-atom Lennard-Jones fcc crystal (64^3 unit cells, density 0.8442,
rc 2.5, skin 0.3, T 0.72, dt 0.005), FP32-pair/FP64-accumulate path versus the
plain FP64 path, with the mixed path's force error against the FP64 reference.

Prints ONE JSON line.  `value` is the mixed path's atom-steps/s with inputs
resident in HBM; the FP64 path's figure, the force error, energy drift, the
event-timed roofline of the dominant kernel and the CPU reference timed on the
host's cores ride along in the same line.

  python bench.py [--steps K] [--warmup W] [--gpus 1]
  python bench.py --copy-probe      # plain 1 GiB device copy (counter calibration)
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0            # MI355X HBM3E, datasheet
# vector ALU: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3 T lane-ops/s (an FMA is one
# op; = the 78.6 TFLOP/s binary64 vector peak counted in FMAs)
ALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# algorithmic lane-ops of the LJ pair loop: every listed pair 9 (displacement 3,
# r^2 5, cutoff test 1); a pair inside rc 17 more (1/r^2 1, q2 1, q6 2, q12 1,
# 2 q12 - q6 2, f_s 2, V 2, force accumulation 3, energy 1, virial 2)
OPS_LISTED, OPS_INSIDE, OPS_ENERGY = 9, 12, 5
FORCE_SOURCES = ["paper_1305_4196_amd/csrc/md_force.hip", "paper_1305_4196_amd/csrc/md_brick.h",
                 "paper_1305_4196_amd/csrc/md_internal.h", "paper_1305_4196_amd/csrc/md_reduce.h"]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def source_hash(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def copy_probe():
    import torch
    n = (1 << 30) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": a.numel() * 8, "copy_probe_bytes_written": b.numel() * 8,
                      "launches": 5}))


def cpu_baseline(w, steps: int):
    """The CPU reference (single-threaded C, binary64) on the first `steps` steps
    of the same run, including its initial list build."""
    import oracle
    t0 = time.perf_counter()
    oracle.verlet(w.pos, w.vel, w.boxes[0], w.pot, w.dt, w.mass, steps, w.skin)
    dt = time.perf_counter() - t0
    return {"value": w.n * steps / dt, "unit": "atom-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} steps of the same {w.n:,}-atom run from its initial state, "
                      f"including the oracle's initial neighbour-list build ({dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--cpu-steps", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true")
    ap.add_argument("--cap", type=int, default=0, help="LDS candidates per cell task")
    ap.add_argument("--wgpc", type=int, default=0)
    ap.add_argument("--brick", type=str, default="", help="brick shape bx,by,bz (cells per task)")
    ap.add_argument("--threads", type=int, default=0, help="threads per brick task")
    ap.add_argument("--shell", action="store_true",
                    help="half lists over 14 of the 27 cells (the 3x3x2 task overlap)")
    ap.add_argument("--tune", action="store_true", help="run the autotuner before timing")
    ap.add_argument("--thermo", type=int, default=100,
                    help="record E_pot, KE, W every this many steps (and after the last)")
    ap.add_argument("--list", choices=["full", "half", "waves", "deps"], default="full",
                    help="full list (each atom written by its own lane), Newton-3 half list with atomics, "
                         "the half list run in waves of non-overlapping brick tasks, "
                         "or the same tasks in dependence order in one persistent launch")
    ap.add_argument("--only", choices=["mixed", "fp64"], default=None,
                    help="time one path only (for profiler runs)")
    ap.add_argument("--workload", default="lj_fcc_1048576",
                    choices=["lj_fcc_1048576", "lj_cluster_slab", "fs_eam_1418342", "replicas_lj_512",
                             "replicas_eam_512"],
                    help="the default is the headline workload; the others print their own line")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              f"(the multi-GPU decomposition is design-only)", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe()
        return

    import numpy as np
    import torch
    from paper_1305_4196_amd import binding as B
    from paper_1305_4196_amd import workloads as W
    from paper_1305_4196_amd.system import MDSystem

    torch.cuda.set_device(0)
    if args.workload.startswith("replicas_"):
        bench_batch(args, args.workload.split("_")[1])
        return
    if args.workload != "lj_fcc_1048576":
        bench_other(args, args.workload)
        return
    w = W.lj_bulk()
    n = w.n
    log(f"workload {w.name}: N={n}, L={w.boxes[0, 0]:.4f}, steps={args.steps}, warmup={args.warmup}")
    sysm = MDSystem.from_workload(w)
    if args.cap:
        B.md_set_tuning(sysm.ctx, 0, args.cap)
    if args.wgpc:
        B.md_set_tuning(sysm.ctx, 1, args.wgpc)
    if args.brick:
        bx, by, bz = (int(v) for v in args.brick.split(","))
        B.md_set_tuning(sysm.ctx, 3, bx | by << 8 | bz << 16)
    if args.threads:
        B.md_set_tuning(sysm.ctx, 4, args.threads)
    if args.shell:
        B.md_set_tuning(sysm.ctx, 6, 1)
    pos0 = torch.tensor(w.pos, dtype=torch.float64, device="cuda")
    vel0 = torch.tensor(w.vel, dtype=torch.float64, device="cuda")
    F = torch.empty_like(pos0)
    hist = torch.zeros(((args.steps + args.thermo - 1) // args.thermo, 3), dtype=torch.float64, device="cuda")
    nreb = torch.zeros(1, dtype=torch.int32, device="cuda")

    results = {}
    kind = {"full": B.MD_LIST_FULL, "half": B.MD_LIST_HALF, "waves": B.MD_LIST_WAVES,
            "deps": B.MD_LIST_DEPS}[args.list]
    paths = [("mixed", B.MD_MIXED), ("fp64", B.MD_FP64)]
    if args.only:
        paths = [p for p in paths if p[0] == args.only]
    for name, prec in paths:
        sysm.pos.copy_(pos0)
        sysm.vel.copy_(vel0)
        B.md_build_cells(sysm.ctx, sysm.pos, sysm.boxes, w.pot.rc, w.skin)
        if args.warmup > 0:
            B.md_verlet_step(sysm.ctx, sysm.dpot, prec, kind, sysm.pos, sysm.vel, F,
                             w.dt, w.mass, args.warmup, None, None)
        code = B.md_get_status(sysm.ctx)[0]
        if code != B.MD_OK:
            raise RuntimeError(f"warm-up ended with status {code}")
        torch.cuda.synchronize()
        B.md_profile(sysm.ctx, True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        B.md_verlet_step(sysm.ctx, sysm.dpot, prec, kind, sysm.pos, sysm.vel, F,
                         w.dt, w.mass, args.steps, hist, nreb, hist_every=args.thermo)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        fms, fn, lms, ln = B.md_profile(sysm.ctx, False)
        code, flags, cap = B.md_get_status(sysm.ctx)
        if code != B.MD_OK:
            raise RuntimeError(f"{name} run ended with status {code} (flags {flags})")
        h = hist.cpu().numpy()
        etot = h[:, 0] + h[:, 1]
        tuning = {"brick": B.md_query(sysm.ctx, 3), "threads": B.md_query(sysm.ctx, 4),
                  "lds_candidates": B.md_query(sysm.ctx, 0), "row_capacity": B.md_query(sysm.ctx, 2),
                  "bricks": B.md_query(sysm.ctx, 5), "grid": B.md_query(sysm.ctx, 9),
                  "max_halo": B.md_query(sysm.ctx, 6), "max_brick_atoms": B.md_query(sysm.ctx, 7),
                  "waves": B.md_query(sysm.ctx, 11), "half_rule": "14-cell" if B.md_query(sysm.ctx, 13) else "sorted"}
        tuning["brick"] = "x".join(str((tuning["brick"] >> s) & 255) for s in (0, 8, 16))
        nbar = B.md_query(sysm.ctx, 10) / n
        # share of the entries stored in 16 bits (the rest take 32)
        narrow = B.md_query(sysm.ctx, 15) / max(nbar * n, 1)
        results[name] = dict(
            seconds=t1 - t0, atom_steps=n * args.steps / (t1 - t0), rebuilds=int(nreb.item()),
            force_ms_avg=fms / max(fn, 1), force_launches=fn, list_ms_total=lms, list_launches=ln,
            nbar=nbar, narrow=narrow, drift=float(np.max(np.abs(etot - etot[0])) / abs(etot[0])),
            T_end=float(2 * h[-1, 1] / (3 * n - 3)), capacity=cap, tuning=tuning)
        log(f"{name}: {results[name]['atom_steps'] / 1e9:.3f} G atom-steps/s, "
            f"{1e3 * (t1 - t0) / args.steps:.3f} ms/step, force kernel {results[name]['force_ms_avg'] * 1e3:.1f} us, "
            f"rebuilds {results[name]['rebuilds']}, nbar {nbar:.2f}, drift {results[name]['drift']:.2e}, "
            f"list {lms / max(ln, 1) * 1e3:.1f} us/launch, tuning {tuning}")

    # force error of the mixed path against the binary64 reference on a thermal snapshot
    import oracle
    snap = W.thermal_snapshot(w, 0.05)
    s2 = MDSystem(snap, w.boxes, w.offsets, w.pot, w.skin)
    Fm = s2.forces(B.MD_MIXED)[0].cpu().numpy()
    Fd = s2.forces(B.MD_FP64)[0].cpu().numpy()
    sample = np.random.default_rng(7).choice(n, size=512, replace=False).astype(np.int32)
    Fo, _ = oracle.lj_atoms(snap, w.boxes[0], sample, w.pot.eps, w.pot.sigma, w.pot.rc)
    err_mixed = float(np.linalg.norm(Fm[:, sample] - Fo) / np.linalg.norm(Fo))
    # listed and interacting pairs of the sampled atoms (minimum image, binary64)
    st_, nb_ = B.md_get_neighbor_list(s2.ctx)
    L = w.boxes[0]
    listed = inside = 0
    for u in sample:
        js = nb_[st_[u]:st_[u + 1]]
        d = snap[:, js] - snap[:, u:u + 1]
        d -= L[:, None] * np.round(d / L[:, None])
        r2 = (d * d).sum(axis=0)
        listed += js.size
        inside += int((r2 < w.pot.rc ** 2).sum())
    inside_frac = inside / max(listed, 1)
    err_fp64 = float(np.linalg.norm(Fd[:, sample] - Fo) / np.linalg.norm(Fo))
    log(f"force error vs reference (512 sampled atoms): mixed {err_mixed:.2e}, fp64 {err_fp64:.2e}")

    main_name = "mixed" if "mixed" in results else "fp64"
    r = results[main_name]
    # The fused LJ force kernel is bound by vector ALU issue, not HBM: its
    # algorithmic lane-ops per atom-step are OPS_LISTED per listed pair plus
    # OPS_INSIDE per pair inside rc, plus OPS_ENERGY per pair inside rc on the
    # steps that record energies; its algorithmic bytes per atom-step are
    # list 2 nbar (16-bit entries; 4 for any entry kept in 32 bits) + x read 24
    # + v read/write 48 + x' write 24 + x_ref read 24.
    t_s = r["force_ms_avg"] * 1e-3
    nbar = r["nbar"]
    ops_per_atom = OPS_LISTED * nbar + (OPS_INSIDE + OPS_ENERGY / args.thermo) * nbar * inside_frac
    bytes_per_atom = (2.0 * r["narrow"] + 4.0 * (1.0 - r["narrow"])) * nbar + 120.0
    achieved_alu = n * ops_per_atom / t_s / 1e12
    achieved_hbm = n * bytes_per_atom / t_s / 1e9
    traffic = None
    tf = os.path.join(ROOT, "profiles", "traffic_lj_force.json")
    if os.path.exists(tf):
        with open(tf) as f:
            t = json.load(f)
        if t.get("source_hash") == source_hash(FORCE_SOURCES) and t.get("path") == main_name:
            traffic = t.get("hbm_bytes_per_launch")
    roofline = {"bound": "alu", "achieved": round(achieved_alu, 3), "peak": round(ALU_PEAK_TOPS, 2),
                "unit": "T lane-ops/s", "frac": round(achieved_alu / ALU_PEAK_TOPS, 4), "traffic": traffic,
                "kernel": "k_lj_full (brick-task LJ forces + velocity Verlet, fused)",
                "kernel_avg_us": round(r["force_ms_avg"] * 1e3, 2),
                "ops_per_atom_step": round(ops_per_atom, 1), "inside_rc_fraction": round(inside_frac, 4),
                "hbm": {"achieved": round(achieved_hbm, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved_hbm / HBM_PEAK_GBS, 4),
                        "bytes_per_atom_step": round(bytes_per_atom, 1),
                        "list_entries_16bit": round(r["narrow"], 4)}}

    line = {
        "metric": "atom-steps/s (forces+neighbor rebuild), FP32-mixed vs FP64 path at stated error",
        "value": round(r["atom_steps"], 1),
        "unit": "atom-steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * r["seconds"] / args.steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32-pair/f64-accumulate" if main_name == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": "lj_fcc_1048576", "atoms": n, "cells": "64^3 fcc", "density": 0.8442,
                   "rc": 2.5, "skin": 0.3, "T": 0.72, "dt": 0.005, "list": args.list, "thermo_every": args.thermo,
                   "parallelism": "single GPU"},
        "fp64_path": ({"value": round(results["fp64"]["atom_steps"], 1),
                       "ms_per_step": round(1e3 * results["fp64"]["seconds"] / args.steps, 4),
                       "force_kernel_us": round(results["fp64"]["force_ms_avg"] * 1e3, 2),
                       "alu_frac": round(n * ops_per_atom / (results["fp64"]["force_ms_avg"] * 1e-3) / 1e12
                                         / ALU_PEAK_TOPS, 4),
                       "hbm_frac": round(n * bytes_per_atom / (results["fp64"]["force_ms_avg"] * 1e-3) / 1e9
                                         / HBM_PEAK_GBS, 4),
                       "energy_drift": results["fp64"]["drift"], "rebuilds": results["fp64"]["rebuilds"]}
                      if "fp64" in results else None),
        "mixed_force_rel_err": err_mixed,
        "fp64_force_rel_err": err_fp64,
        "energy_drift": r["drift"],
        "rebuilds": r["rebuilds"],
        "mean_neighbors": round(r["nbar"], 3),
        "list_ms_total": round(r["list_ms_total"], 3),
        "tuning": r["tuning"],
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        log("timing the CPU reference ...")
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_steps)
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)


def _tune(B, sysm, args):
    if args.cap:
        B.md_set_tuning(sysm.ctx, 0, args.cap)
    if args.wgpc:
        B.md_set_tuning(sysm.ctx, 1, args.wgpc)
    if args.brick:
        bx, by, bz = (int(v) for v in args.brick.split(","))
        B.md_set_tuning(sysm.ctx, 3, bx | by << 8 | bz << 16)
    if args.threads:
        B.md_set_tuning(sysm.ctx, 4, args.threads)
    if args.tune:
        from paper_1305_4196_amd import tune
        best = tune.tune(sysm, precision=B.MD_MIXED)
        log(f"tuned: brick {best['shape']} on {best['threads']} threads ({best['ms']:.3f} ms per force + "
            f"amortised build)")


def bench_other(args, name):
    """atom-steps/s of md_verlet_step on the inhomogeneous LJ system or the EAM
    crystal, both paths, with the force error of the mixed path."""
    import numpy as np
    import torch
    import oracle
    from paper_1305_4196_amd import binding as B
    from paper_1305_4196_amd import workloads as W
    from paper_1305_4196_amd.system import MDSystem

    w = W.WORKLOADS[name]()
    n = w.n
    steps = args.steps if args.steps != 1000 or name != "fs_eam_1418342" else w.steps
    log(f"workload {w.name}: N={n}, steps={steps}, warmup={args.warmup}")
    sysm = MDSystem.from_workload(w)
    _tune(B, sysm, args)
    pos0 = torch.tensor(w.pos, dtype=torch.float64, device="cuda")
    vel0 = torch.tensor(w.vel, dtype=torch.float64, device="cuda")
    F = torch.empty_like(pos0)
    hist = torch.zeros(((steps + args.thermo - 1) // args.thermo, 3), dtype=torch.float64, device="cuda")
    nreb = torch.zeros(1, dtype=torch.int32, device="cuda")
    res = {}
    for pname, prec in (("mixed", B.MD_MIXED), ("fp64", B.MD_FP64)):
        if args.only and args.only != pname:
            continue
        # a run whose lists overflow is repeated from the same state once the
        # context has grown the rows (the documented capacity protocol)
        for attempt in range(4):
            sysm.pos.copy_(pos0)
            sysm.vel.copy_(vel0)
            B.md_build_cells(sysm.ctx, sysm.pos, sysm.boxes, w.pot.rc, w.skin)
            if args.warmup:
                B.md_verlet_step(sysm.ctx, sysm.dpot, prec, B.MD_LIST_FULL, sysm.pos, sysm.vel, F, w.dt,
                                 w.mass, args.warmup, None, None)
            torch.cuda.synchronize()
            B.md_profile(sysm.ctx, True)
            t0 = time.perf_counter()
            B.md_verlet_step(sysm.ctx, sysm.dpot, prec, B.MD_LIST_FULL, sysm.pos, sysm.vel, F, w.dt, w.mass,
                             steps, hist, nreb, hist_every=args.thermo)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            fms, fn, lms, ln = B.md_profile(sysm.ctx, False)
            code = B.md_get_status(sysm.ctx)[0]
            if code != B.MD_ERR_CAPACITY:
                break
            log(f"{pname}: list rows overflowed, repeating with capacity {B.md_query(sysm.ctx, 2)}")
        if code != B.MD_OK:
            raise RuntimeError(f"{pname} run ended with status {code}")
        h = hist.cpu().numpy()
        et = h[:, 0] + h[:, 1]
        res[pname] = {"atom_steps_per_s": round(n * steps / (t1 - t0), 1),
                      "ms_per_step": round(1e3 * (t1 - t0) / steps, 4),
                      "force_us": round(1e3 * fms / max(fn, 1), 2), "rebuilds": int(nreb.item()),
                      "list_ms_total": round(lms, 3),
                      "energy_drift": float(np.max(np.abs(et - et[0])) / max(abs(et[0]), 1e-300)),
                      "mean_neighbors": round(B.md_query(sysm.ctx, 10) / n, 3),
                      "brick": B.md_query(sysm.ctx, 3), "threads": B.md_query(sysm.ctx, 4)}
        log(f"{pname}: {res[pname]}")
    # force error of the mixed path on a thermal snapshot
    snap = W.thermal_snapshot(w, 0.05)
    s2 = MDSystem(snap, w.boxes, w.offsets, w.pot, w.skin)
    Fm = s2.forces(B.MD_MIXED)[0].cpu().numpy()
    L = w.boxes[0]
    if w.pot.kind == "lj":
        sample = np.random.default_rng(7).choice(n, size=512, replace=False).astype(np.int32)
        Fo, _ = oracle.lj_atoms(snap, L, sample, w.pot.eps, w.pot.sigma, w.pot.rc)
        err = float(np.linalg.norm(Fm[:, sample] - Fo) / np.linalg.norm(Fo))
    else:
        Fo, _, _ = oracle.forces(oracle.wrap(snap, L), L, w.pot, skin=w.skin)
        err = float(np.linalg.norm(Fm - Fo) / np.linalg.norm(Fo))
    main = res.get("mixed") or res.get("fp64")
    print(json.dumps({"metric": "atom-steps/s (forces+neighbor rebuild), FP32-mixed vs FP64 path at stated error",
                      "value": main["atom_steps_per_s"], "unit": "atom-steps/s", "n_gpus": 1, "steps": steps,
                      "warmup": args.warmup, "ms_per_step": main["ms_per_step"], "higher_is_better": True,
                      "data": "synthetic", "config": {"workload": w.name, "atoms": n, "thermo_every": args.thermo},
                      "paths": res,
                      "mixed_force_rel_err": err}), flush=True)


def bench_batch(args, kind):
    """Gradient evaluations per second of the 512-replica fitting batch (forces,
    loss cotangent and adjoint replayed as one graph), with the oracle's
    forward + adjoint timed on a sample of the replicas."""
    import numpy as np
    import torch
    import oracle
    from paper_1305_4196_amd import binding as B
    from paper_1305_4196_amd import workloads as W
    from paper_1305_4196_amd.fit import BatchedFit
    from paper_1305_4196_amd.system import MDSystem

    w = W.replica_batch(kind, 512)
    n = w.n
    log(f"workload {w.name}: {w.n_replicas} replicas, N={n}")
    sysm = MDSystem.from_workload(w)
    _tune(B, sysm, args)
    F_star = sysm.forces(B.MD_FP64)[0]
    start = W.perturb_params(w.pot)
    if kind == "lj":
        theta = torch.tensor([start.eps, start.sigma], dtype=torch.float64, device="cuda")
    else:
        theta = torch.tensor(np.concatenate([start.phi.coef.ravel(), start.rho.coef.ravel(),
                                             start.embed.coef.ravel()]), dtype=torch.float64, device="cuda")
    fit = BatchedFit(sysm, F_star, theta)
    fit.capture()
    for _ in range(max(args.warmup, 3)):
        fit.gradient()
    torch.cuda.synchronize()
    reps = max(args.steps // 10, 20)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fit.gradient()
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) * 1e-3 / reps
    if B.md_get_status(sysm.ctx)[0] != B.MD_OK:
        raise RuntimeError("batch run ended with a device error")
    log(f"graph replay {t * 1e3:.3f} ms per batch gradient, loss {fit.loss():.4e}")
    line = {"metric": "batch gradients/s (forces + adjoint over the replica batch, one graph replay)",
            "value": round(1.0 / t, 2), "unit": "batch-gradients/s", "n_gpus": 1,
            "replica_gradients_per_s": round(w.n_replicas / t, 1), "atom_gradients_per_s": round(n / t, 1),
            "ms_per_batch_gradient": round(t * 1e3, 4), "higher_is_better": True, "dtype": "f64",
            "data": "synthetic", "config": {"workload": w.name, "replicas": w.n_replicas, "atoms": n,
                                            "params": int(theta.numel())}}
    if not args.no_cpu_baseline:
        log("timing the CPU reference on 32 replicas ...")
        F_np = F_star.cpu().numpy()
        t0 = time.perf_counter()
        for r in range(32):
            lo, hi = int(w.offsets[r]), int(w.offsets[r + 1])
            L = w.boxes[r]
            x = oracle.wrap(w.pos[:, lo:hi], L)
            Fr, _, _ = oracle.forces(x, L, start, skin=w.skin)
            u = 2.0 * (Fr - F_np[:, lo:hi]) / (3.0 * n)
            oracle.vjp(x, L, start, u, 0.0, skin=w.skin)
        dt = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": round(32 / dt, 3), "unit": "replica-gradients/s", "cores": 1,
                                "kind": "oracle", "sample": f"forward + adjoint of replicas 0..31 ({dt:.1f} s)"}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
