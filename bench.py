"""Benchmark: the foaming lattice sweep on the 384^3 D3Q19 + D3Q7 power-law foam with
2000 bubbles (synthetic, seeded), on one MI355X.

A step is one pass of the whole hot path: lattice sweep, cell conversion, bubble
labelling and gas bookkeeping, bubble pressures, curvature and disjoining pressure.
Two runs: (i) populations stored in binary32 with the plain paraboloid-fit curvature
("FP32 plain") and (ii) populations stored as binary16 offsets f_i - w_i with binary32
arithmetic and the learned curvature closure (plain fit as fallback). ``value`` is the
whole-step MLUPS of run (ii); run (i) and the ratio are reported beside it. The network
of run (ii) is trained on the GPU by the library before the timed region (2M generated
stencils by default), and its training time and validation error are reported.

The same binary16 + learned-curvature run is repeated under gravity (a body force along
-z, reported under ``body_force``) and with a Carreau-Yasuda liquid (``carreau_yasuda``); the
metric's workload itself is a power-law liquid without body force.

A third measurement covers the batched ensemble (48 independent domains of 64^3 to 160^3,
binary16 storage, learned curvature): MLUPS over all domains stepped one after another,
and with the tuned bulk sweep and one launch per kernel for all domains, overlapped as in
a single domain's step.

The roofline entry is the bulk sweep kernel: algorithmic bytes per launch over its
average duration inside the timed steps, measured with events on its stream; there it
shares the GPU with the previous step's labelling and geometry, which run on a second
stream. ``roofline.isolated`` times the same kernel launched alone, back to back. Before
each timed window the library's tuner picks the bulk kernel's launch shape on the live
state (untimed).

After its timed window the reported run advances to step 2000 and times the same number
of steps there (``late_state``: the bubbles have grown, more cells are interface and gas).
``accuracy_vs_oracle`` compares the production form with the FP64 oracle on a 96^3 crop of
the same recipe (liquid-mass drift, bubble-volume error). ``cpu_baseline`` runs the
single-threaded oracle on that crop, once alone and as one copy per host core.

Prints one JSON line. Options: --gpus N (only 1), --steps K, --warmup W,
--workload NAME, --no-cpu-baseline, --mlp-train N, --mlp-epochs E, --no-ensemble,
--ensemble-steps S, --late-steps L, --accuracy-steps A.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# Counter-derived HBM traffic of the bulk sweep, valid only for the sources it was taken on.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_sweep_vec_c3_foam_384_traffic.md")
TRAFFIC_SOURCES = ("paper_1908_04262_amd/csrc/sweep_impl.h",
                   "paper_1908_04262_amd/csrc/sweep_f16.hip",
                   "paper_1908_04262_amd/csrc/sweep_f32.hip",
                   "paper_1908_04262_amd/csrc/mf_internal.h",
                   "paper_1908_04262_amd/build.py")


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE/WRITE_SIZE summary
    (already scaled by the copy-kernel calibration), or None when the summary is missing or
    the sweep sources have changed since the counters were taken."""
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    h = hashlib.sha256()
    for rel in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    m = re.search(r"source_sha256: ([0-9a-f]{64})", text)
    if not m or m.group(1) != h.hexdigest():
        return None
    m = re.search(r"traffic_bytes_per_launch " + re.escape(kernel) + r": (\d+)", text)
    return int(m.group(1)) if m else None
METRIC = "MLUPS & %HBM peak, 384^3 foam; FP16-store+MLP-curvature vs FP32 plain"
# launch shapes of the bulk sweep (cells per thread, threads per work-group), by variant
VARIANTS = [(4, 256), (2, 256), (4, 128), (2, 128), (8, 256), (8, 128), (8, 64), (4, 64)]


BYTES_F = {"fp64": 8, "fp32": 4, "f16s": 2, "bf16s": 2, "f16s_g16": 2}
BYTES_G = {"fp64": 8, "fp32": 4, "f16s": 4, "bf16s": 4, "f16s_g16": 2}


def bytes_per_fluid_cell(wl, prec):
    """Algorithmic bytes of one fluid-cell update: each population read once and written
    once (f: Q values, g: Qg values) plus the cell's type byte."""
    Q, Qg = (9, 5) if wl["dim"] == 2 else (19, 7)
    return 2 * Q * BYTES_F[prec] + 2 * Qg * BYTES_G[prec] + 1


def plain_cells(T, dim):
    """Liquid cells with no wall among their lattice neighbours: the cells the bulk
    sweep kernel updates (interface and near-wall cells go to the list kernel)."""
    import numpy as np
    W = T == 3
    nw = np.zeros_like(W)
    dirs = [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)
            if 0 < abs(a) + abs(b) + abs(c) <= 2]
    if dim == 2:
        dirs = [(0, b, c) for (a, b, c) in dirs if a == 0]
    pad = np.pad(W, 1, constant_values=False)
    nz, ny, nx = T.shape
    for (dz, dy, dx) in dirs:
        nw |= pad[1 + dz:1 + dz + nz, 1 + dy:1 + dy + ny, 1 + dx:1 + dx + nx]
    return int(np.count_nonzero((T == 2) & ~nw))


def sweep_bytes(wl, T, prec):
    """Algorithmic bytes of one launch of the bulk sweep kernel: every plain liquid cell
    costs a full update, every other cell its type byte."""
    per_cell = bytes_per_fluid_cell(wl, prec)
    n_plain = plain_cells(T, wl["dim"])
    return n_plain * per_cell + (int(T.size) - n_plain), n_plain, per_cell


def train_net(n_train, epochs, log):
    import torch

    from paper_1908_04262_amd import CurvatureNet

    n_val = max(4096, n_train // 16)
    net = CurvatureNet(7)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rmse = net.train(n_train=n_train, n_val=n_val, epochs=epochs, batch=4096, lr=2e-3, data_seed=4)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    log(f"[mlp] trained on {n_train} stencils x {epochs} epochs in {dt:.1f}s, val rmse {rmse:.4f}")
    return net, dict(n_train=n_train, n_val=n_val, epochs=epochs, seconds=round(dt, 2),
                     val_rmse_kappa=round(rmse, 5))


def time_field_nucleation(wl, log):
    """Host time of the Poisson-disk nucleation sampler on the benchmark grid: the liquid
    region filled with sites of radius U[2, 4] at least r_i + r_j + 1 apart, then thinned by a
    field that rises linearly along x from 0.1 to 1, keeping up to 2000 sites."""
    import numpy as np

    from paper_1908_04262_amd import poisson_nuclei

    nx, ny, nz = wl["nx"], wl["ny"], wl["nz"]
    P = np.broadcast_to(np.linspace(0.1, 1.0, nx, dtype=np.float32), (nz, ny, nx))
    t0 = time.perf_counter()
    c, r = poisson_nuclei(wl, P, 2000, 2.0, 4.0, 1.0, 30, wl["seed"])
    dt = time.perf_counter() - t0
    log(f"[nucleation] {len(r)} sites from the field in {dt:.2f}s")
    return {"sites": int(len(r)), "seconds": round(dt, 3), "grid": [nx, ny, nz], "r": [2.0, 4.0],
            "field": "linear in x from 0.1 to 1", "host": True}


def late_window(sim, wl, until, steps, log):
    """Advance the foam to step `until` and time `steps` more steps there: the bubbles have
    grown, so more cells are interface and gas than in the first window."""
    import numpy as np
    import torch

    done = sim.ledgers()["step"]
    t0 = time.perf_counter()
    while done < until:
        n = min(500, until - done)
        sim.step(n)
        sim.sync()
        done += n
        log(f"[{wl['precision']}] late state: step {done}")
    adv = time.perf_counter() - t0
    sim.profile(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t1
    sim.sync()
    bulk_ms, nsw = sim.profile_get(0)
    spec_ms, _ = sim.profile_get(2)
    sim.profile(False)
    T = sim.read("type")
    led = sim.ledgers()
    ncell = int(np.prod(sim.shape))
    out = dict(step=int(done), steps=steps, mlups=round(ncell * steps / wall / 1e6, 2),
               ms_per_step=round(wall * 1e3 / steps, 4), bulk_sweep_ms=round(bulk_ms / max(nsw, 1), 4),
               special_sweep_ms=round(spec_ms / max(nsw, 1), 4),
               interface_fraction=round(float(np.count_nonzero(T == 1)) / ncell, 5),
               gas_fraction=round(float(np.count_nonzero(T == 0)) / ncell, 5),
               n_bubbles=led["n_bubbles"], advance_seconds=round(adv, 2), status=led["status"])
    log(f"[{wl['precision']}] late state {json.dumps(out)}")
    return out


def run_one(wl, steps, warmup, log, net=None, late_steps=0):
    import numpy as np
    import torch

    from paper_1908_04262_amd import Sim
    from synth import place_nuclei

    t0 = time.time()
    sim = Sim(wl, device=0)
    if net is not None:
        sim.attach_mlp(net)
    c, r, p0 = place_nuclei(wl)
    sim.nucleate(c, r, p0)
    log(f"[{wl['precision']}] created + nucleated {len(r)} nuclei in {time.time() - t0:.1f}s")
    sim.step(warmup)
    sim.sync()
    # the project's tuner picks the bulk-sweep launch shape on the live state (untimed)
    variant, tune_ms = sim.tune(5)
    log(f"[{wl['precision']}] warmup {warmup} steps done; tuned bulk-sweep shape {variant} "
        f"({[round(float(x), 3) for x in tune_ms]} ms)")
    T0 = sim.read("type")
    bytes0, np0, per_cell = sweep_bytes(wl, T0, wl["precision"])
    sim.profile(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    sim.sync()
    bulk_ms, nsw = sim.profile_get(0)
    step_ms, nst = sim.profile_get(1)
    spec_ms, _ = sim.profile_get(2)
    sim.profile(False)
    T1 = sim.read("type")
    bytes1, np1, _ = sweep_bytes(wl, T1, wl["precision"])
    # the bulk kernel alone (back-to-back launches on the final state, nothing beside it):
    # inside the step it shares the GPU with the previous step's labelling and geometry
    _, tune_ms = sim.tune(20)
    sim.set_sweep_variant(variant)
    iso_ms = float(tune_ms[variant])
    led = sim.ledgers()
    ncell = int(np.prod(sim.shape))
    wall = t2 - t1
    bulk_avg_s = bulk_ms / 1e3 / max(nsw, 1)
    bytes_launch = 0.5 * (bytes0 + bytes1)
    n_fluid = int(np.count_nonzero((T1 == 1) | (T1 == 2)))
    res = dict(
        precision=wl["precision"],
        curvature=wl["curvature"],
        mlups=ncell * steps / wall / 1e6,
        ms_per_step=wall * 1e3 / steps,
        bulk_sweep_ms=bulk_avg_s * 1e3,
        special_sweep_ms=spec_ms / max(nsw, 1),
        step_event_ms=step_ms / max(nst, 1),
        bulk_sweep_bytes=bytes_launch,
        bulk_sweep_gbs=bytes_launch / bulk_avg_s / 1e9,
        bulk_isolated_ms=iso_ms,
        bulk_isolated_gbs=bytes1 / (iso_ms / 1e3) / 1e9 if iso_ms > 0 else None,
        bytes_per_fluid_cell=per_cell,
        n_plain=0.5 * (np0 + np1),
        n_fluid=n_fluid,
        n_interface=int(np.count_nonzero(T1 == 1)),
        n_bubbles=led["n_bubbles"],
        status=led["status"],
    )
    # whole-step algorithmic HBM fraction: full-update bytes of every fluid cell per step
    # over the wall time of a step
    step_bytes = n_fluid * per_cell + (ncell - n_fluid)
    res["hbm_frac_step"] = step_bytes / (wall / steps) / 1e9 / HBM_PEAK_GBS
    res["bulk_variant"] = int(variant)
    if late_steps > 0:
        res["late_state"] = late_window(sim, wl, late_steps, steps, log)
    log(f"[{wl['precision']}/{wl['curvature']}] {json.dumps(res)}")
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return res


def run_ensemble(net, steps, log, until=0):
    """The batched ensemble (48 domains of 64^3..160^3, binary16 storage, learned
    curvature): MLUPS over all domains when every domain is stepped in turn, and with the
    tuned bulk sweep and one launch per kernel for all domains."""
    import numpy as np
    import torch

    from paper_1908_04262_amd import Batch, Sim
    from synth import batch_workloads, place_nuclei

    wls = batch_workloads()
    t0 = time.time()
    sims = []
    for wl in wls:
        s = Sim(wl, device=0)
        s.attach_mlp(net)
        s.nucleate(*place_nuclei(wl))
        sims.append(s)
    cells = int(sum(np.prod(s.shape) for s in sims))
    for s in sims:
        s.step(2)
    torch.cuda.synchronize()
    log(f"[ensemble] {len(sims)} domains, {cells / 1e6:.1f}M cells, set up in {time.time() - t0:.1f}s")
    t1 = time.perf_counter()
    for _ in range(steps):
        for s in sims:
            s.step(1)
    torch.cuda.synchronize()
    seq = cells * steps / (time.perf_counter() - t1) / 1e6
    batch = Batch(sims)
    variants = batch.tune(3)
    batch.step(2)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    batch.step(steps)
    torch.cuda.synchronize()
    bat = cells * steps / (time.perf_counter() - t2) / 1e6
    long = None
    if until > 0:
        # carry on with the batched launches until every domain has taken `until` steps:
        # liquid mass (plus the lost-liquid ledger) and total gas are conserved quantities
        def conserved(s):
            t = s.ledgers()
            return (t["liquid"] + t["lost_liquid"],
                    t["dissolved"] + t["bubble_gas"] + t["atm_gas"] + t["collapsed_gas"])
        c0 = [conserved(s) for s in sims]
        done = int(sims[0].ledgers()["step"])
        left = max(until - done, 0)
        t3 = time.perf_counter()
        batch.step(left)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t3
        c1 = [conserved(s) for s in sims]
        led = [s.ledgers() for s in sims]
        long = {"steps_per_domain": int(led[0]["step"]), "batched_steps": left,
                "mlups_batched": round(cells * left / dt / 1e6, 1) if left else None,
                "seconds": round(dt, 2),
                "max_rel_liquid_drift": max(abs(b[0] - a[0]) / a[0] for a, b in zip(c0, c1)),
                "max_rel_gas_drift": max(abs(b[1] - a[1]) / a[1] for a, b in zip(c0, c1)),
                "bubbles": int(sum(t["n_bubbles"] for t in led)),
                "all_at_step": all(int(t["step"]) == int(led[0]["step"]) for t in led)}
        log(f"[ensemble] {left} more batched steps to step {long['steps_per_domain']}: "
            f"{long['mlups_batched']} MLUPS, {json.dumps(long)}")
    st = [s.ledgers()["status"] for s in sims]
    log(f"[ensemble] sequential {seq:.0f} MLUPS, batched {bat:.0f} MLUPS, variants "
        f"{dict(zip(*np.unique(variants, return_counts=True)))}")
    batch.close()
    for s in sims:
        s.close()
    del sims
    torch.cuda.empty_cache()
    return {"domains": len(wls), "cells": cells, "steps": steps,
            "mlups_sequential": round(seq, 1), "mlups_batched": round(bat, 1),
            "speedup": round(bat / seq, 3), "status_ok": all(x == 0 for x in st),
            "tuned_variants": [int(v) for v in variants], "long_run": long}


def crop_workload(n=96):
    """the 384^3 recipe (power-law foam, supersaturation 1.5, r ~ U[2,4]) on an n^3 crop
    with the same bubble density"""
    from synth import workload

    frac = (n / 384.0) ** 3
    wl = workload("c3_foam_384", nx=n, ny=n, nz=n, precision="fp64", max_ids=4096)
    wl["gas_from"] = int(0.75 * n)
    wl["nuclei"] = dict(wl["nuclei"], n=max(1, int(round(2000 * frac))))
    return wl


def _oracle_crop_rate(args):
    """one process: the oracle on the crop for `steps` steps; returns seconds"""
    n, steps = args
    from oracle import Oracle
    from synth import place_nuclei

    wl = crop_workload(n)
    o = Oracle(wl)
    o.nucleate(*place_nuclei(wl))
    t0 = time.perf_counter()
    o.step(steps)
    return time.perf_counter() - t0


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(log, budget_s=10.0):
    """The FP64 oracle on the host on a 96^3 crop of the benchmark recipe: first one
    process (the oracle is single-threaded), then one independent copy per host core (at
    most 16, the machine's CPU share), each on the same crop; the aggregate rate of the copies
    is the value."""
    import multiprocessing as mp

    n = 96
    ncell = n ** 3
    t1 = _oracle_crop_rate((n, 4))
    steps = max(2, min(50, int(budget_s / max(t1 / 4, 1e-3))))
    single = ncell * 4 / t1 / 1e6
    cores = max(1, min(16, os.cpu_count() or 1))
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(cores) as pool:
        secs = pool.map(_oracle_crop_rate, [(n, steps)] * cores)
    wall = time.perf_counter() - t0
    agg = cores * ncell * steps / max(secs) / 1e6
    log(f"cpu baseline: 1 process {single:.3f} MLUPS; {cores} processes x {steps} steps of {n}^3 "
        f"in {wall:.1f}s -> {agg:.3f} MLUPS ({cpu_model()})")
    return dict(value=agg, unit="MLUPS", cores=cores, kind="oracle",
                single_thread_value=single, cpu_model=cpu_model(),
                sample=f"{cores} independent single-threaded FP64 oracle processes, {steps} steps each of a "
                       f"{n}^3 crop of the 384^3 recipe ({crop_workload(n)['nuclei']['n']} nuclei); the "
                       f"oracle itself is single-threaded")


def crop_accuracy(net, steps, log):
    """Error of the production form (binary16 f and g, learned curvature) against the FP64
    oracle on the 96^3 crop: relative liquid-mass drift and the largest relative bubble
    volume deviation, over `steps` steps (compared only while the oracle's bubble ids are
    unchanged)."""
    import numpy as np

    from oracle import Oracle
    from paper_1908_04262_amd import Sim
    from synth import place_nuclei

    wl64 = crop_workload(96)
    wl = dict(wl64, precision="f16s_g16", curvature="mlp")
    gpu = Sim(wl)
    gpu.attach_mlp(net)
    orc = Oracle(wl64)
    c, r, p0 = place_nuclei(wl64)
    gpu.nucleate(c, r, p0)
    orc.nucleate(c, r, p0)
    t0 = gpu.totals()
    m0 = t0["liquid"] + t0["lost_liquid"]
    worst_v, worst_m, compared, done = 0.0, 0.0, 0, 0
    chunk = max(1, steps // 5)
    while done < steps:
        gpu.step(chunk)
        orc.step(chunk)
        done += chunk
        t = gpu.totals()
        worst_m = max(worst_m, abs(t["liquid"] + t["lost_liquid"] - m0) / m0)
        bg, bo = gpu.bubbles(), orc.bubbles()
        if list(bg["id"]) == list(bo["id"]) and bo["id"].size:
            worst_v = max(worst_v, float((np.abs(bg["V"] - bo["V"]) / bo["V"]).max()))
            compared += 1
    gpu.close()
    out = dict(steps=done, mass_drift=worst_m, max_volume_error=worst_v, comparisons=compared,
               crop="96^3 crop of the 384^3 recipe", reference="FP64 oracle, plain curvature")
    log(f"[accuracy] {json.dumps(out)}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="c3_foam_384")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mlp-train", type=int, default=1966080)
    ap.add_argument("--mlp-epochs", type=int, default=8)
    ap.add_argument("--late-steps", type=int, default=2000)
    ap.add_argument("--accuracy-steps", type=int, default=25)
    ap.add_argument("--no-ensemble", action="store_true")
    ap.add_argument("--ensemble-steps", type=int, default=20)
    ap.add_argument("--ensemble-until", type=int, default=0,
                    help="continue the batched ensemble until every domain has taken this many steps")
    ap.add_argument("--quiet", action="store_true")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py runs on one GPU only: mifoam has no multi-GPU path "
              "(a domain would shard by z-slabs; that path is not built).", file=sys.stderr)
        sys.exit(2)

    def log(msg):
        if not a.quiet:
            print(msg, file=sys.stderr, flush=True)

    from synth import workload

    wl = workload(a.workload)
    r32 = run_one(dict(wl, precision="fp32", curvature="plain"), a.steps, a.warmup, log)
    net, train_info = train_net(a.mlp_train, a.mlp_epochs, log)
    r16 = run_one(dict(wl, precision="f16s_g16", curvature="mlp"), a.steps, a.warmup, log, net=net,
                  late_steps=a.late_steps)
    r16f = run_one(dict(wl, precision="f16s", curvature="mlp"), a.steps, a.warmup, log, net=net)
    # the same foam under gravity (body-force term, forced kernel instances)
    grav = (0.0, 0.0, -3e-5)
    r16g = run_one(dict(wl, precision="f16s_g16", curvature="mlp", accel=grav), max(a.steps // 2, 1),
                   a.warmup, log, net=net)
    # the same foam with a Carreau-Yasuda liquid (shear thinning between tau_inf and tau0)
    cy = dict(rheology="carreau_yasuda", cy_tau0=1.2, cy_tau_inf=0.6, cy_lambda=1000.0, cy_a=2.0, cy_n=0.4)
    r16c = run_one(dict(wl, precision="f16s_g16", curvature="mlp", **cy), max(a.steps // 2, 1),
                   a.warmup, log, net=net)
    nuc = time_field_nucleation(wl, log)
    ens = None if a.no_ensemble else run_ensemble(net, a.ensemble_steps, log, a.ensemble_until)
    cpu = None if a.no_cpu_baseline else cpu_baseline(log)
    acc = None if a.accuracy_steps <= 0 else crop_accuracy(net, a.accuracy_steps, log)

    def brief(r):
        return {"mlups": round(r["mlups"], 2), "ms_per_step": round(r["ms_per_step"], 4),
                "hbm_frac_step": round(r["hbm_frac_step"], 4),
                "bulk_sweep_gbs": round(r["bulk_sweep_gbs"], 1),
                "bulk_sweep_ms": round(r["bulk_sweep_ms"], 4),
                "special_sweep_ms": round(r["special_sweep_ms"], 4),
                "bulk_variant": r["bulk_variant"], "status": r["status"]}

    out = {
        "metric": METRIC,
        "value": round(r16["mlups"], 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(r16["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{wl['name']}: {wl['nx']}x{wl['ny']}x{wl['nz']} D3Q19+D3Q7 power-law "
                        f"foam, {wl['nuclei']['n']} bubbles r~U[2,4], seed {wl['seed']}",
            "storage": "f and g as binary16 offsets, binary32 arithmetic (value); "
                       "binary32 (fp32_plain)",
            "curvature": "learned 125-64-64-1 MLP with plain-fit fallback (value); "
                         "plain fit (fp32_plain)",
        },
        "mlp_training": train_info,
        "hbm_frac_step": round(r16["hbm_frac_step"], 4),
        "status": r16["status"],
        "fp32_plain": brief(r32),
        "f16_f_only_mlp": brief(r16f),
        "body_force": dict(brief(r16g), accel=list(grav), steps=max(a.steps // 2, 1)),
        "carreau_yasuda": dict(brief(r16c), params={k: v for k, v in cy.items() if k != "rheology"},
                               steps=max(a.steps // 2, 1)),
        "speedup_vs_fp32_plain": round(r16["mlups"] / r32["mlups"], 3),
        "late_state": r16.get("late_state"),
        "accuracy_vs_oracle": acc,
        "roofline": {
            "bound": "hbm",
            "kernel": f"k_sweep_vec<3,4,{VARIANTS[r16['bulk_variant']][0]},{VARIANTS[r16['bulk_variant']][1]}> "
                      "(bulk sweep, binary16 f and g)",
            "achieved": round(r16["bulk_sweep_gbs"], 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(r16["bulk_sweep_gbs"] / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(f"k_sweep_vec<3,4,{VARIANTS[r16['bulk_variant']][0]},"
                                        f"{VARIANTS[r16['bulk_variant']][1]}>"),
            "bytes_per_launch": r16["bulk_sweep_bytes"],
            "avg_launch_ms": round(r16["bulk_sweep_ms"], 4),
            "isolated": {"achieved": round(r16["bulk_isolated_gbs"], 1),
                         "frac": round(r16["bulk_isolated_gbs"] / HBM_PEAK_GBS, 4),
                         "avg_launch_ms": round(r16["bulk_isolated_ms"], 4)},
        },
        "field_nucleation": nuc,
        "batched_ensemble": ens,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
