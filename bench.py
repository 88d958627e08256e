#!/usr/bin/env python3
"""Throughput of the MD hot path on one MI355X.

The headline is atom-steps/s of velocity Verlet (forces + device-decided
neighbour rebuilds + integration + energy sums) on the 1,048,576-atom
Lennard-Jones fcc crystal (64^3 unit cells, density 0.8442, rc 2.5, skin 0.3,
T 0.72, dt 0.005), FP32-pair/FP64-accumulate path (`value`) beside the plain
FP64 path.  The timed region is the step loop of md_verlet_step with its inputs
resident in HBM: HIP events around the loop, recorded by the library on its
stream, so the setup of the call (user order to sorted, cells, first list,
F(x0)) is left out, as the paper leaves out initialisation (Sec. III); the
host wall clock around the whole call is reported beside it.

The same JSON line carries:
  - energy drift over the timed steps (the energies at the start of the timed
    run are row 0), rebuilds, mean list length, force error of both paths
    against the oracle on sampled atoms of a thermal snapshot;
  - the step loop with energies recorded on every step;
  - the roofline of the dominant kernel (the fused LJ force + integration
    kernel on steps without energy terms): algorithmic bytes 4 nbar + 120 per
    atom-step against 8 TB/s, algorithmic lane-ops 35 per pair inside rc and
    9 per listed pair beyond it against 39.3 T lane-ops/s, the larger fraction
    named as the bound;
  - the oracle timed on the host (one core; and the OpenMP full-list variant on
    all the cores the process may use), setup subtracted;
  - the other workloads: the 256-atom crystal (us/step), the inhomogeneous
    cluster + voided slab, the 1.4M-atom FS-EAM crystal, and the 512-replica
    fitting batches (gradients/s).

  python bench.py [--steps K] [--warmup W] [--gpus 1]
  python bench.py --workload fs_eam_1418342 --steps 100   # one workload only
  python bench.py --copy-probe      # plain 1 GiB device copy (counter calibration)
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "atom-steps/s (forces+neighbor rebuild), FP32-mixed vs FP64 path at stated error"
HBM_PEAK_GBS = 8000.0            # MI355X HBM3E, datasheet
# vector ALU: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3 T lane-ops/s (an FMA is one
# op; = the 78.6 TFLOP/s binary64 vector peak counted in FMAs)
ALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# algorithmic work of the LJ full-list step per atom: bytes 4 nbar (list, 32-bit
# entries) + 120 (x read 24, v read+write 48, x' write 24, x_ref read 24);
# lane-ops 35 per pair inside rc, 9 per listed pair beyond it
LJ_OPS_INSIDE, LJ_OPS_LISTED = 35, 9
FORCE_SOURCES = ["paper_1305_4196_amd/csrc/md_force.hip", "paper_1305_4196_amd/csrc/md_brick.h",
                 "paper_1305_4196_amd/csrc/md_internal.h", "paper_1305_4196_amd/csrc/md_reduce.h"]
EXTRA_WORKLOADS = ["lj_fcc_256", "lj_cluster_slab", "fs_eam_1418342", "replicas_lj_512", "replicas_eam_512"]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def code_only(text: str) -> str:
    """C/C++ source without its comments, runs of whitespace collapsed: what the compiler
    reads (a comment edit leaves the kernels, and so their counters, unchanged)."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c in "\"'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def source_hash(paths):
    """Hash of the code (comments excluded) of the sources the force kernel is built from."""
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), encoding="utf-8") as f:
            h.update(code_only(f.read()).encode())
    return h.hexdigest()[:16]


def host_threads() -> int:
    """Cores this process may use: OMP_NUM_THREADS when set, else the affinity mask."""
    env = os.environ.get("OMP_NUM_THREADS", "")
    n = len(os.sched_getaffinity(0))
    if env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


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


# ---------------------------------------------------------------------- CPU baselines
def cpu_baseline(w, steps: int, threads: int):
    """The oracle on `steps` steps of the run from its initial state, minus a
    0-step run (wrap, first list build, F(x0)); threads = 0 is the serial
    reference, threads >= 1 the OpenMP full-list variant."""
    import oracle
    t0 = time.perf_counter()
    oracle.verlet(w.pos, w.vel, w.boxes[0], w.pot, w.dt, w.mass, 0, w.skin, threads=threads)
    t1 = time.perf_counter()
    _, _, _, _, nreb = oracle.verlet(w.pos, w.vel, w.boxes[0], w.pot, w.dt, w.mass, steps, w.skin,
                                     threads=threads)
    t2 = time.perf_counter()
    dt = max((t2 - t1) - (t1 - t0), 1e-9)
    kind = "serial, half lists" if threads == 0 else f"OpenMP on {threads} threads, full lists"
    return {"value": round(w.n * steps / dt, 1), "unit": "atom-steps/s", "cores": max(threads, 1),
            "kind": "oracle",
            "sample": f"{steps} velocity-Verlet steps of the same {w.n:,}-atom run from its initial state "
                      f"({nreb} list rebuilds among them), {kind}; its setup (wrap, first list, F(x0)), "
                      f"timed as a 0-step run ({t1 - t0:.1f} s), subtracted from the {t2 - t1:.1f} s run"}


# ---------------------------------------------------------------------- one MD workload
def tune_system(B, sysm, args, precision, w=None):
    """Brick shape and workgroup size: fixed by the flags, else the autotuner's."""
    if args.brick or args.threads:
        if args.brick:
            bx, by, bz = (int(v) for v in args.brick.split(","))
            B.md_set_tuning(sysm.ctx, 3, bx | by << 8 | bz << 16)
        if args.threads:
            B.md_set_tuning(sysm.ctx, 4, args.threads)
        return {"source": "flags"}
    if args.no_tune:
        return {"source": "occupancy heuristic"}
    from paper_1305_4196_amd import tune
    best = tune.tune(sysm, precision=precision, dt=w.dt if w is not None else 0.005,
                     mass=w.mass if w is not None else 1.0)
    log(f"tuned: brick {best['shape']} on {best['threads']} threads "
        f"({best['ms'] * 1e3:.1f} us per step)")
    return {"source": "autotuner", "shape": "x".join(str(v) for v in best["shape"]), "threads": best["threads"],
            "candidates": [{"shape": "x".join(str(v) for v in c["shape"]), "threads": c["threads"],
                            "us": round(c["ms"] * 1e3, 1)} for c in best.get("candidates", [])]}


def run_md(B, torch, sysm, w, prec, kind, steps, warmup, thermo, pos0, vel0):
    """One timed md_verlet_step run of `steps` steps after `warmup` steps.
    A run whose lists overflow is repeated from the same state once the context
    has grown the rows (the documented capacity protocol)."""
    import numpy as np
    n = w.n
    F = torch.empty_like(pos0)
    rows = (steps + thermo - 1) // thermo
    hist = torch.zeros((rows, 3), dtype=torch.float64, device="cuda")
    nreb = torch.zeros(1, dtype=torch.int32, device="cuda")
    E0 = torch.zeros(1, dtype=torch.float64, device="cuda")
    for attempt in range(4):
        sysm.pos.copy_(pos0)
        sysm.vel.copy_(vel0)
        B.md_build_cells(sysm.ctx, sysm.pos, sysm.boxes, w.pot.rc, w.skin)
        if warmup > 0:
            B.md_verlet_step(sysm.ctx, sysm.dpot, prec, kind, sysm.pos, sysm.vel, F, w.dt, w.mass, warmup,
                             None, None)
        code = B.md_get_status(sysm.ctx)[0]
        if code == B.MD_ERR_CAPACITY:
            continue
        if code != B.MD_OK:
            raise RuntimeError(f"warm-up ended with status {code}")
        # energies at the start of the timed run (row 0 of the drift)
        B.md_build_cells(sysm.ctx, sysm.pos, sysm.boxes, w.pot.rc, w.skin)
        B.md_build_neighbor_list(sysm.ctx, B.MD_LIST_FULL)
        B.md_compute_forces(sysm.ctx, sysm.dpot, prec, F, E0, None)
        ke0 = 0.5 * w.mass * float((sysm.vel * sysm.vel).sum().item())
        x_start, v_start = sysm.pos.clone(), sysm.vel.clone()
        torch.cuda.synchronize()
        # the timed run: events at the ends of the setup and of the step loop only
        B.md_profile(sysm.ctx, True, launches=False)
        t0 = time.perf_counter()
        B.md_verlet_step(sysm.ctx, sysm.dpot, prec, kind, sysm.pos, sysm.vel, F, w.dt, w.mass, steps, hist,
                         nreb, hist_every=thermo)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        B.md_profile(sysm.ctx, False)
        det = B.md_profile_detail(sysm.ctx)
        code, flags, cap = B.md_get_status(sysm.ctx)
        if code != B.MD_ERR_CAPACITY:
            break
        log(f"list rows overflowed, repeating with capacity {B.md_query(sysm.ctx, 2)}")
    if code != B.MD_OK:
        raise RuntimeError(f"run ended with status {code} (flags {flags})")
    # the same run again with an event pair around every force and list launch
    # (per-launch durations; the pairs themselves slow the loop a little)
    x_end, v_end = sysm.pos.clone(), sysm.vel.clone()
    sysm.pos.copy_(x_start)
    sysm.vel.copy_(v_start)
    hist2 = torch.zeros_like(hist)
    B.md_profile(sysm.ctx, True)
    B.md_verlet_step(sysm.ctx, sysm.dpot, prec, kind, sysm.pos, sysm.vel, F, w.dt, w.mass, steps, hist2,
                     None, hist_every=thermo)
    fms, fn, lms, ln = B.md_profile(sysm.ctx, False)
    det_l = B.md_profile_detail(sysm.ctx)
    code2 = B.md_get_status(sysm.ctx)[0]
    if code2 != B.MD_OK:
        raise RuntimeError(f"instrumented run ended with status {code2}")
    sysm.pos.copy_(x_end)
    sysm.vel.copy_(v_end)
    h = hist.cpu().numpy()
    e0 = float(E0.item()) + ke0
    etot = np.concatenate([[e0], h[:, 0] + h[:, 1]])
    loop_s = det["loop_ms"] * 1e-3
    nbar = B.md_query(sysm.ctx, 10) / n
    narrow = B.md_query(sysm.ctx, 15) / max(nbar * n, 1)
    shape = B.md_query(sysm.ctx, 3)
    out = {
        "atom_steps_per_s": round(n * steps / loop_s, 1),
        "ms_per_step": round(1e3 * loop_s / steps, 5),
        "wall_atom_steps_per_s": round(n * steps / (t1 - t0), 1),
        "setup_ms": round(det["setup_ms"], 3),
        "instrumented_ms_per_step": round(det_l["loop_ms"] / max(det_l["loop_steps"], 1), 5),
        "force_plain_us": round(1e3 * det_l["force_plain_ms"] / det_l["force_plain_n"], 2) if det_l["force_plain_n"] else None,
        "force_plain_launches": det_l["force_plain_n"],
        "force_energy_us": round(1e3 * det_l["force_energy_ms"] / det_l["force_energy_n"], 2) if det_l["force_energy_n"] else None,
        "force_energy_launches": det_l["force_energy_n"],
        "list_ms_total": round(lms, 3), "list_launches": ln,
        "rebuilds": int(nreb.item()),
        "energy_drift": float(np.max(np.abs(etot - etot[0])) / max(abs(etot[0]), 1e-300)),
        "energy_rows": int(etot.size), "thermo_every": thermo,
        "T_end": float(2 * h[-1, 1] / (3 * n - 3)),
        "mean_neighbors": round(nbar, 3), "list_entries_16bit": round(narrow, 4),
        "brick": "x".join(str((shape >> s) & 255) for s in (0, 8, 16)), "threads": B.md_query(sysm.ctx, 4),
        "sched": "queue" if B.md_query(sysm.ctx, 14) == 2 else "static",
    }
    return out


def force_errors(B, np, oracle, W, MDSystem, w, n_sample=512):
    """Relative force error (S14) of both paths against the oracle on a thermal
    snapshot (every force vanishes on the perfect lattice): LJ on sampled atoms
    (exhaustive per-atom oracle), EAM on the whole system."""
    snap = W.thermal_snapshot(w, 0.05)
    s2 = MDSystem(snap, w.boxes, w.offsets, w.pot, w.skin)
    Fm = s2.forces(B.MD_MIXED)[0].cpu().numpy()
    Fd = s2.forces(B.MD_FP64)[0].cpu().numpy()
    L = w.boxes[0]
    out = {}
    if w.pot.kind == "lj":
        sample = np.random.default_rng(7).choice(w.n, size=min(n_sample, w.n), replace=False).astype(np.int32)
        Fo, _ = oracle.lj_atoms(snap, L, sample, w.pot.eps, w.pot.sigma, w.pot.rc)
        Fm, Fd = Fm[:, sample], Fd[:, sample]
        out["sample"] = f"{sample.size} atoms"
        # listed and interacting pairs of the sampled atoms (for the roofline's lane-ops)
        st, nb = B.md_get_neighbor_list(s2.ctx)
        listed = inside = 0
        for u in sample:
            js = nb[st[u]:st[u + 1]]
            d = snap[:, js] - snap[:, u:u + 1]
            d -= L[:, None] * np.round(d / L[:, None])
            listed += js.size
            inside += int(((d * d).sum(axis=0) < w.pot.rc ** 2).sum())
        out["inside_rc_fraction"] = inside / max(listed, 1)
    else:
        Fo, _, _ = oracle.forces(oracle.wrap(snap, L), L, w.pot, skin=w.skin)
        out["sample"] = "all atoms"
    frms = math.sqrt(float(np.mean(np.sum(Fo * Fo, axis=0))))
    for name, Fg in (("mixed", Fm), ("fp64", Fd)):
        out[name] = float(np.linalg.norm(Fg - Fo) / np.linalg.norm(Fo))
        out[name + "_max_atom_over_rms"] = float(np.max(np.sqrt(np.sum((Fg - Fo) ** 2, axis=0))) / frms)
    return out


def bench_md(args, name, steps, warmup, thermo, paths=("mixed", "fp64"), errors=True, tune=True,
             per_step_energy=False):
    import numpy as np
    import torch
    import oracle
    from paper_1305_4196_amd import binding as B
    from paper_1305_4196_amd import workloads as W
    from paper_1305_4196_amd.system import MDSystem

    w = W.WORKLOADS[name]()
    log(f"workload {w.name}: N={w.n}, steps={steps}, warmup={warmup}, thermo every {thermo}")
    sysm = MDSystem.from_workload(w)
    if args.cap:
        B.md_set_tuning(sysm.ctx, 0, args.cap)
    if args.wgpc:
        B.md_set_tuning(sysm.ctx, 1, args.wgpc)
    if args.shell:
        B.md_set_tuning(sysm.ctx, 6, 1)
    prec_of = {"mixed": B.MD_MIXED, "fp64": B.MD_FP64}
    tuning = tune_system(B, sysm, args, prec_of[paths[0]], w) if tune else {"source": "occupancy heuristic"}
    kind = {"full": B.MD_LIST_FULL, "half": B.MD_LIST_HALF, "waves": B.MD_LIST_WAVES,
            "deps": B.MD_LIST_DEPS}[args.list]
    pos0 = torch.tensor(w.pos, dtype=torch.float64, device="cuda")
    vel0 = torch.tensor(w.vel, dtype=torch.float64, device="cuda")
    res = {"atoms": w.n, "steps": steps, "tuning": tuning}
    for pname in paths:
        r = run_md(B, torch, sysm, w, prec_of[pname], kind, steps, warmup, thermo, pos0, vel0)
        res[pname] = r
        log(f"{name} {pname}: {r['atom_steps_per_s'] / 1e9:.3f} G atom-steps/s ({r['ms_per_step']:.4f} ms/step "
            f"loop, {r['wall_atom_steps_per_s'] / 1e9:.3f} G with setup), force {r['force_plain_us']} us plain / "
            f"{r['force_energy_us']} us recorded, rebuilds {r['rebuilds']}, nbar {r['mean_neighbors']}, "
            f"drift {r['energy_drift']:.2e}")
    if per_step_energy:
        r = run_md(B, torch, sysm, w, prec_of[paths[0]], kind, steps, warmup, 1, pos0, vel0)
        res[paths[0] + "_energy_every_step"] = r
        log(f"{name} {paths[0]}, energies every step: {r['atom_steps_per_s'] / 1e9:.3f} G atom-steps/s, "
            f"force {r['force_energy_us']} us")
    if errors:
        res["force_rel_err"] = force_errors(B, np, oracle, W, MDSystem, w)
        log(f"{name} force error vs oracle: {res['force_rel_err']}")
    return w, res


def roofline_lj(w, res, path, traffic):
    """Roofline of the fused LJ full-list kernel on steps without energy terms."""
    r = res[path]
    t_s = r["force_plain_us"] * 1e-6
    nbar = r["mean_neighbors"]
    fin = res["force_rel_err"]["inside_rc_fraction"]
    bytes_alg = 4.0 * nbar + 120.0
    ops = LJ_OPS_INSIDE * nbar * fin + LJ_OPS_LISTED * nbar * (1.0 - fin)
    hbm = w.n * bytes_alg / t_s / 1e9
    alu = w.n * ops / t_s / 1e12
    hbm_frac, alu_frac = hbm / HBM_PEAK_GBS, alu / ALU_PEAK_TOPS
    narrow = r["list_entries_16bit"]
    bytes_stored = (2.0 * narrow + 4.0 * (1.0 - narrow)) * nbar + 120.0
    hbm_side = {"bound": "hbm", "achieved": round(hbm, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(hbm_frac, 4), "bytes_per_atom_step": round(bytes_alg, 1)}
    alu_side = {"bound": "alu", "achieved": round(alu, 3), "peak": round(ALU_PEAK_TOPS, 2), "unit": "T lane-ops/s",
                "frac": round(alu_frac, 4), "lane_ops_per_atom_step": round(ops, 1)}
    main, other = (hbm_side, alu_side) if hbm_frac >= alu_frac else (alu_side, hbm_side)
    out = dict(main)
    out.update({"traffic": traffic,
                "kernel": "k_lj_full<" + ("mixed" if path == "mixed" else "fp64") +
                          ", no energy terms> (brick-task LJ forces + velocity Verlet, fused)",
                "kernel_avg_us": r["force_plain_us"], "launches": r["force_plain_launches"],
                "inside_rc_fraction": round(fin, 4), "other_bound": other,
                "stored_list_view": {"bytes_per_atom_step": round(bytes_stored, 1),
                                     "list_entries_16bit": narrow,
                                     "achieved": round(w.n * bytes_stored / t_s / 1e9, 1), "unit": "GB/s"}})
    return out


def bench_batch(args, kind, reps=None, cpu=True):
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
    if args.brick or args.threads:
        tune_system(B, sysm, args, B.MD_FP64)
    F_star = sysm.forces(B.MD_FP64)[0]
    start = W.perturb_params(w.pot)
    if kind == "lj":
        theta = torch.tensor([start.eps, start.sigma], dtype=torch.float64, device="cuda")
    else:
        theta = torch.tensor(np.concatenate([start.phi.coef.ravel(), start.rho.coef.ravel(),
                                             start.embed.coef.ravel()]), dtype=torch.float64, device="cuda")
    fit = BatchedFit(sysm, F_star, theta, tune=not (args.brick or args.threads or args.no_tune))
    if fit.tuning is not None:
        log(f"{w.name}: tuned brick {fit.tuning['shape']} on {fit.tuning['threads']} threads "
            f"({fit.tuning['ms'] * 1e3:.1f} us per forces + adjoint)")
    fit.capture()
    for _ in range(3):
        fit.gradient()
    torch.cuda.synchronize()
    reps = reps or 50
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fit.gradient()
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) * 1e-3 / reps
    if B.md_get_status(sysm.ctx)[0] != B.MD_OK:
        raise RuntimeError("batch run ended with a device error")
    log(f"{w.name}: graph replay {t * 1e3:.3f} ms per batch gradient, loss {fit.loss():.4e}")
    out = {"batch_gradients_per_s": round(1.0 / t, 2), "replica_gradients_per_s": round(w.n_replicas / t, 1),
           "atom_gradients_per_s": round(n / t, 1), "ms_per_batch_gradient": round(t * 1e3, 4),
           "replicas": w.n_replicas, "atoms": n, "params": int(theta.numel()), "dtype": "f64", "replays": reps,
           "tuning": ({"source": "autotuner (forces + adjoint)",
                       "shape": "x".join(str(v) for v in fit.tuning["shape"]), "threads": fit.tuning["threads"],
                       "candidates": [{"shape": "x".join(str(v) for v in c["shape"]), "threads": c["threads"],
                                       "us": round(c["ms"] * 1e3, 1)} for c in fit.tuning.get("candidates", [])]}
                      if fit.tuning is not None else {"source": "flags or occupancy heuristic"})}
    if cpu:
        m = 16
        F_np = F_star.cpu().numpy()
        t0 = time.perf_counter()
        for r in range(m):
            lo, hi = int(w.offsets[r]), int(w.offsets[r + 1])
            L = w.boxes[r]
            x = oracle.wrap(w.pos[:, lo:hi], L)
            Fr, _, _ = oracle.forces(x, L, start, skin=w.skin)
            u = 2.0 * (Fr - F_np[:, lo:hi]) / (3.0 * n)
            oracle.vjp(x, L, start, u, 0.0, skin=w.skin)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(m / dt, 3), "unit": "replica-gradients/s", "cores": 1,
                               "kind": "oracle", "sample": f"forward + adjoint of replicas 0..{m - 1} ({dt:.1f} s)"}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--cpu-steps", type=int, default=16, help="steps of the single-core oracle baseline")
    ap.add_argument("--cpu-steps-all", type=int, default=40, help="steps of the all-cores oracle baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="the headline workload only")
    ap.add_argument("--no-tune", action="store_true", help="occupancy heuristic instead of the autotuner")
    ap.add_argument("--copy-probe", action="store_true")
    ap.add_argument("--cap", type=int, default=0, help="LDS candidates per cell task")
    ap.add_argument("--wgpc", type=int, default=0)
    ap.add_argument("--brick", type=str, default="", help="brick shape bx,by,bz (cells per task)")
    ap.add_argument("--threads", type=int, default=0, help="threads per brick task")
    ap.add_argument("--shell", action="store_true",
                    help="half lists over 14 of the 27 cells (the 3x3x2 task overlap)")
    ap.add_argument("--thermo", type=int, default=100,
                    help="record E_pot, KE, W every this many steps (at most steps/10) and after the last")
    ap.add_argument("--list", choices=["full", "half", "waves", "deps"], default="full",
                    help="full list (each atom written by its own lane), Newton-3 half list with atomics, "
                         "the half list run in waves of non-overlapping brick tasks, "
                         "or the same tasks in dependence order in one persistent launch")
    ap.add_argument("--only", choices=["mixed", "fp64"], default=None,
                    help="time one path only (for profiler runs)")
    ap.add_argument("--workload", default="lj_fcc_1048576",
                    choices=["lj_fcc_1048576", "lj_fcc_256", "lj_cluster_slab", "fs_eam_1418342",
                             "replicas_lj_512", "replicas_eam_512"],
                    help="the default is the headline workload (with the others as extra keys); "
                         "another name prints that workload's line only")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              f"(the multi-GPU decomposition is design-only)", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe()
        return

    import tempfile
    import torch
    torch.cuda.set_device(0)
    # the autotuner's choices of this run only (a cache from another build of the
    # kernels would not apply)
    os.environ["MD_TUNE_CACHE"] = os.path.join(tempfile.mkdtemp(prefix="md_tune_"), "tune.json")
    thermo = max(1, min(args.thermo, args.steps // 10 if args.steps >= 10 else 1))
    paths = (args.only,) if args.only else ("mixed", "fp64")

    if args.workload.startswith("replicas_"):
        res = bench_batch(args, args.workload.split("_")[1], reps=max(args.steps // 10, 20),
                          cpu=not args.no_cpu_baseline)
        print(json.dumps({"metric": "batch gradients/s (forces + adjoint over the replica batch, one graph replay)",
                          "value": res["batch_gradients_per_s"], "unit": "batch-gradients/s", "n_gpus": 1,
                          "higher_is_better": True, "data": "synthetic",
                          "config": {"workload": args.workload}, **res}), flush=True)
        return
    if args.workload != "lj_fcc_1048576":
        w, res = bench_md(args, args.workload, args.steps, args.warmup, thermo, paths=paths,
                          tune=not args.workload == "lj_fcc_256")
        main_r = res[paths[0]]
        print(json.dumps({"metric": METRIC, "value": main_r["atom_steps_per_s"], "unit": "atom-steps/s",
                          "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                          "ms_per_step": main_r["ms_per_step"], "higher_is_better": True, "data": "synthetic",
                          "config": {"workload": w.name, "atoms": w.n, "thermo_every": thermo}, **res}),
              flush=True)
        return

    # ------------------------------------------------------------------ headline
    w, res = bench_md(args, "lj_fcc_1048576", args.steps, args.warmup, thermo, paths=paths,
                      per_step_energy=True)
    main_name = paths[0]
    r = res[main_name]
    traffic = None
    tf = os.path.join(ROOT, "profiles", "traffic_lj_force.json")
    if os.path.exists(tf):
        with open(tf) as f:
            recs = json.load(f).get("records", [])
        # counters taken on the same kernel sources, path and launch shape only
        for t in recs:
            if (t.get("source_hash") == source_hash(FORCE_SOURCES) and t.get("path") == main_name
                    and t.get("brick") == r["brick"] and t.get("threads") == r["threads"]):
                traffic = t.get("hbm_bytes_per_launch")
    roof = roofline_lj(w, res, main_name, traffic)
    other_paths = {p: res[p] for p in paths if p != main_name}
    line = {
        "metric": METRIC,
        "value": r["atom_steps_per_s"],
        "unit": "atom-steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32-pair/f64-accumulate" if main_name == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": "lj_fcc_1048576", "atoms": w.n, "cells": "64^3 fcc", "density": 0.8442,
                   "rc": 2.5, "skin": 0.3, "T": 0.72, "dt": 0.005, "list": args.list, "thermo_every": thermo,
                   "parallelism": "single GPU"},
        "timed_region": "md_verlet_step's step loop (one HIP event at each end, on its stream); setup excluded, reported beside; per-launch durations from a second run of the same steps with an event pair around every launch (instrumented_ms_per_step)",
        "energy_drift": r["energy_drift"],
        "rebuilds": r["rebuilds"],
        "mean_neighbors": r["mean_neighbors"],
        "force_rel_err": res["force_rel_err"],
        "run": r,
        "other_path": other_paths,
        "energy_every_step": res.get(main_name + "_energy_every_step"),
        "tuning": res["tuning"],
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        log("timing the CPU reference (one core) ...")
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_steps, 0)
        nt = host_threads()
        log(f"timing the CPU reference (OpenMP, {nt} threads) ...")
        line["cpu_baseline_all_cores"] = cpu_baseline(w, args.cpu_steps_all, nt)
    else:
        line["cpu_baseline"] = None

    if not args.no_extras:
        extras = {}
        # the workload's own length (1,000 steps) when the timed run is shorter
        if args.steps < 1000:
            _, full = bench_md(args, "lj_fcc_1048576", 1000, args.warmup, 100, paths=paths, errors=False)
            extras["lj_fcc_1048576_1000_steps"] = {p: full[p] for p in paths}
        _, small = bench_md(args, "lj_fcc_256", 100, 10, 10, paths=("fp64", "mixed"), errors=False, tune=False)
        for p in ("fp64", "mixed"):
            small[p]["us_per_step"] = round(1e3 * small[p]["ms_per_step"], 2)
        if not args.no_cpu_baseline:
            import oracle
            from paper_1305_4196_amd import workloads as W
            ws = W.lj_small()
            t0 = time.perf_counter()
            oracle.verlet(ws.pos, ws.vel, ws.boxes[0], ws.pot, ws.dt, ws.mass, 100, ws.skin)
            small["cpu_baseline"] = {"value": round(ws.n * 100 / (time.perf_counter() - t0), 1),
                                     "unit": "atom-steps/s", "cores": 1, "kind": "oracle",
                                     "sample": "all 100 steps, setup included"}
        extras["lj_fcc_256"] = small
        _, extras["lj_cluster_slab"] = bench_md(args, "lj_cluster_slab", 1000, args.warmup, 100, paths=paths)
        _, extras["fs_eam_1418342"] = bench_md(args, "fs_eam_1418342", 500, args.warmup, 50, paths=paths)
        extras["replicas_lj_512"] = bench_batch(args, "lj", cpu=not args.no_cpu_baseline)
        extras["replicas_eam_512"] = bench_batch(args, "eam", cpu=not args.no_cpu_baseline)
        line["workloads"] = extras
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
