"""Benchmark: RF-CMP EFIE solve on one MI355X.

One step = one pass of the whole hot path over the workload, from the mesh
to the RWG currents:
  PEC sphere r = 1 m, icosphere level 4 (C = 5120 cells, N = 7680 RWG),
  ka = 1.0 and ka = 1e-4, one x-polarised plane wave along +z, CG to 1e-6:
  topology, projector matrices (L^+, G_ll^-1), far/near-pair assembly of T_A
  and V, power-iteration scalings, excitation, preconditioned rhs, CG, and
  recovery j = P_o i -- for both wavenumbers.

Prints one JSON line.  ``value`` = RF-CMP solves per second over the timed
steps (two solves per step); kernel durations come from HIP events recorded
by the library on the launch stream during the timed steps.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

import synth  # noqa: E402

# MI355X published peaks
HBM_GBS = 8000.0
FP32_VALU_TFLOPS = 157.3
FP64_VALU_TFLOPS = 78.6

WORKLOAD = {"workload": "PEC sphere r=1 m, icosphere level 4 (5120 cells, 7680 RWG), ka=1.0 and ka=1e-4, "
                        "x-polarised plane wave along +z, CG to relative residual 1e-6",
            "mesh": "icosphere4", "ka": [1.0, 1e-4], "nrhs": 1, "tol": 1e-6}
TOL = 1e-6
KS = (1.0, 1e-4)
FAR_FLOPS_PER_POINT_PAIR = 30     # sub 3, R^2 5, rsqrt 1, R 1, kR 1, sin+cos 2, G 3, moment sums 14 (FMA = 2)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-slab", type=int, default=32, help="1/slab of the test cells for the oracle sample")
    p.add_argument("--no-precision-study", action="store_true")
    p.add_argument("--no-spectral-study", action="store_true")
    p.add_argument("--batch-rhs", type=int, default=64)
    p.add_argument("--uneven-batch", action="store_true",
                   help="also time the uneven batch (32 objects x 8 wavenumbers x 4 plane waves, BF16x3), "
                        "through rfcmp_batch_solve and through one rfcmp_solve per operator")
    p.add_argument("--copy-calibration", action="store_true",
                   help="only run a 1 GiB device copy (byte-counter calibration) and exit")
    return p.parse_args()


def cpu_baseline(xyz, tri, slab):
    """The FP64 oracle on a bounded sample of the same workload: its far-pair
    quadrature and near-pair integrals for every slab-th test cell of the
    level-4 sphere at ka = 1.0 (its own functions, row by row, in the order
    its assembly runs them).  Converted to solves/s assuming assembly is the
    oracle's only cost, an upper bound on its throughput: setup, scalings and
    CG are left out."""
    from threadpoolctl import threadpool_limits
    from oracle import assembly, quadrature
    from oracle.topology import Topology
    top = Topology(xyz, tri)
    C = top.C
    rows = np.arange(0, C, slab)
    pts, w = quadrature.tri7_points(top.xyz, top.tri)
    cores = os.cpu_count() or 1
    with threadpool_limits(limits=cores):
        t0 = time.perf_counter()
        c0 = time.process_time()
        near = assembly.near_mask(top)
        k = 1.0
        for s in range(0, len(rows), 8):
            assembly.far_rows(top, k, rows[s:s + 8], pts, w)
        for c in rows:
            for cp in np.nonzero(near[c, c:])[0] + c:
                assembly.near_block(top, c, cp, k, pts, w)
        dt = time.perf_counter() - t0
        used = max(1, int(round((time.process_time() - c0) / dt)))
    pairs = len(rows) * C
    pairs_per_s = pairs / dt
    full_assembly_s = C * C / pairs_per_s
    return {"value": 1.0 / full_assembly_s, "unit": "solves/s", "cores": used,
            "kind": "oracle",
            "sample": f"oracle far+near assembly of 1/{slab} of the test cells ({len(rows)} x {C} cell pairs, "
                      f"ka=1.0) in {dt:.1f} s; solves/s = 1/(C^2 / pairs_per_s), i.e. assembly only "
                      f"(upper bound on the oracle's throughput)",
            "assembly_pairs_per_s": pairs_per_s}


def copy_calibration():
    """A plain device-to-device copy of 1 GiB (5 launches), for scaling the
    HBM byte counters of a profiler run: each launch reads and writes
    exactly 2^30 bytes."""
    import torch
    n = 1 << 30
    a = torch.empty(n, dtype=torch.uint8, device="cuda:0").fill_(1)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_per_launch": n, "launches": 5}))


BF16_MFMA_TFLOPS = 2500.0

# HBM bytes per launch of the symmetric products (k_symv, level-4 sphere) from
# two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE, KiB per dispatch, mean
# over the dispatches of the tag's instantiation), each scaled by what the
# same counter reads for a plain 1 GiB device copy (FETCH_SIZE reads 2^19
# KiB for 2^30 bytes fetched: scale 2.0; WRITE_SIZE reads 2^20 KiB: scale
# 1.0).  Valid only for the kernel source they were taken on: reported as
# null once symv.hip changes.
TRAFFIC_SOURCE = {"path": "paper_1803_08333_amd/csrc/symv.hip",
                  "sha256": "cbdcf6878b657550db4fe78b3d29caab17a48ac76d3c03b83ba5c46ee919e29a"}
TRAFFIC_SCALE = {"fetch": 2.0, "write": 1.0}
TRAFFIC_KIB = {  # tag: (FETCH_SIZE, WRITE_SIZE)
    "cmatvec_ta+v": (174943.0, 5200.1), "cmatvec_ta+v_nr2": (174225.0, 8800.1), "dmatvec_lp": (53270.9, 3200.0),
    "dmatvec_lp_nr2": (53999.6, 6400.0), "dmatvec_lp+gll": (67984.1, 4082.0)}


def measured_traffic(tag):
    import hashlib
    if tag not in TRAFFIC_KIB:
        return None
    src = os.path.join(os.path.dirname(os.path.abspath(__file__)), TRAFFIC_SOURCE["path"])
    with open(src, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != TRAFFIC_SOURCE["sha256"]:
            return None
    fk, wk = TRAFFIC_KIB[tag]
    return 1024.0 * (fk * TRAFFIC_SCALE["fetch"] + wk * TRAFFIC_SCALE["write"])


def _timed_solve(torch, op, e):
    op.solve(e, tol=TOL, maxit=2000)          # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    j, st, info = op.solve(e, tol=TOL, maxit=2000)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3, st, info


def precision_study(rf, torch, nb):
    """BF16x3 (precision 1) against the complex64/FP64 path (precision 0), both
    to the same true relative residual 1e-6, on the workloads the comparison
    is defined on: the level-4 sphere (one plane wave, ka = 1 and 1e-4), the
    jittered 96 x 48 torus (one plane wave, ka = 0.5) and the level-5 sphere
    (nb seeded plane waves, ka = 2), with the BF16x3 T_A product's MFMA and
    HBM rates from HIP events on the last."""
    out = {"tol": TOL}
    kh, pol = synth.default_plane_wave()
    singles = [("icosphere4", synth.icosphere(4), 1.0), ("icosphere4", synth.icosphere(4), 1e-4),
               ("torus96x48", synth.torus(), 0.5)]
    for name, (xyz, tri), k in singles:
        m = rf.Mesh(xyz, tri)
        start = torch.from_numpy(synth.complex_start(m.N, 11)).cuda()
        row = {}
        for prec in (0, 1):
            op = rf.Operator(m, k, power_start=start, precision=prec)
            ms, st, info = _timed_solve(torch, op, op.rhs_planewave(kh, pol))
            row["bf16x3" if prec else "fp32"] = {"solve_ms": ms, "iters": info[0]["iters"],
                                                 "rounds": info[0]["restarts"] + 1,
                                                 "rel_residual": info[0]["rel_residual"], "status": st}
            op.close()
        out[f"{name} ka={k}, 1 rhs"] = row
        m.close()
    xyz, tri = synth.icosphere(5)
    m = rf.Mesh(xyz, tri)
    N = m.N
    start = torch.from_numpy(synth.complex_start(N, 11)).cuda()
    kb, pb = synth.plane_waves(nb, 4)
    row = {}
    for prec in (0, 1):
        op = rf.Operator(m, 2.0, power_start=start, precision=prec)
        e = op.rhs_planewave(kb, pb)
        op.solve(e, tol=TOL, maxit=2000)
        torch.cuda.synchronize()
        rf.profile_select(None)
        rf.profile_enable(True)
        t0 = time.perf_counter()
        j, st, info = op.solve(e, tol=TOL, maxit=2000)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        gt, gn = rf.profile_read("gemm_ta")
        rf.profile_enable(False)
        r = {"solve_ms": ms, "ms_per_rhs": ms / nb, "max_iters": max(i["iters"] for i in info),
             "max_rel_residual": max(i["rel_residual"] for i in info), "status": st}
        if prec == 1 and gn:
            avg = gt / gn
            mfma_flops = 3 * 8.0 * N * N * nb      # three bf16 products per real MAC, 4 real MACs per complex
            r["gemm_ta"] = {"avg_ms": avg, "launches": gn,
                            "mfma_tflops": mfma_flops / (avg * 1e-3) / 1e12,
                            "mfma_frac": mfma_flops / (avg * 1e-3) / 1e12 / BF16_MFMA_TFLOPS,
                            "hbm_gbs": 8.0 * N * N / (avg * 1e-3) / 1e9}
        row["bf16x3" if prec else "fp32"] = r
        op.close()
    out[f"icosphere5 ka=2.0, {nb} rhs"] = row
    m.close()
    return out


def spectral_study(rf):
    """cond(A) of the RF-CMP system against ka (1 down to the 1e-25 Hz of the
    paper's sphere study) on icosphere levels 2-4 and the 96 x 48 torus: the
    CG-Lanczos estimate of a solve of A i = b with a seeded generic b (the
    library's rfcmp_solve_system), power-iteration scalings."""
    from paper_1803_08333_amd import study
    ks = [1.0, 1e-2, 1e-4, 1e-12, study.K_1E_25_HZ]
    meshes = {f"icosphere{L}": synth.icosphere(L) for L in (2, 3, 4)}
    meshes["torus96x48"] = synth.torus()
    rows = study.condition_study(meshes, ks, seed=7)
    out = {}
    for r in rows:
        out.setdefault(r["mesh"], {"N": r["N"], "cond": {}, "iters": {}})
        out[r["mesh"]]["cond"][f"{r['k']:.3g}"] = round(r["cond"], 4)
        out[r["mesh"]]["iters"][f"{r['k']:.3g}"] = r["iters"]
    return out


def far_field_measurement(rf, torch):
    """Far field and bistatic RCS of the library's solution (icosphere level 4,
    x-polarised wave along +z, CG to 1e-8) on the E- and H-plane cuts at 1
    degree (2 x 181 directions): the far-field launch time (HIP events) and,
    at ka = 1e-4, the backscatter RCS against the closed-form Rayleigh limit
    9 pi a^2 (ka)^4 of a small PEC sphere.  (The comparison with the full Mie
    series on the cuts is a GPU test.)"""
    kh, pol = synth.default_plane_wave()
    th = np.linspace(0.0, np.pi, 181)
    d = np.concatenate([np.stack([np.sin(th), np.zeros(181), np.cos(th)], 1),
                        np.stack([np.zeros(181), np.sin(th), np.cos(th)], 1)])
    xyz, tri = synth.icosphere(4)
    m = rf.Mesh(xyz, tri)
    out = {"directions": len(d), "cells": m.C}
    for ka in (1.0, 1e-4):
        op = rf.Operator(m, ka, power_start=torch.from_numpy(synth.complex_start(m.N, 11)).cuda())
        j, st, info = op.solve(op.rhs_planewave(kh, pol), tol=1e-8, maxit=2000)
        op.far_field(j, d)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        _, s = op.far_field(j, d)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b)
        row = {"far_field_ms": ms, "cell_directions_per_s": m.C * len(d) / (ms * 1e-3), "iters": info[0]["iters"],
               "rcs_backscatter": float(s[0, 180].item())}
        if ka < 1e-2:
            row["rayleigh_backscatter"] = 9 * np.pi * ka ** 4
        out[f"ka={ka:g}"] = row
        op.close()
    m.close()
    return out


def voltage_gap_measurement(rf, torch):
    """Voltage-gap source (the Fokker example's second excitation, Sec. 4) on
    the level-4 sphere: a 1 V gap across one edge, CG to 1e-8, iterations and
    solve time at ka = 1 and 1e-4 (the paper reports far fewer iterations for
    its gap source than for its plane wave); at ka = 1 also the power balance
    between the gap's input power Re(V conj(j_m)) and the radiated power of
    the far field over a 24 x 48 Gauss-Legendre x trapezoid direction set."""
    xyz, tri = synth.icosphere(4)
    m = rf.Mesh(xyz, tri)
    gap = 11
    mu, wmu = np.polynomial.legendre.leggauss(24)
    ph = 2 * np.pi * np.arange(48) / 48
    MU, PH = np.meshgrid(mu, ph, indexing="ij")
    d = np.stack([np.sqrt(1 - MU ** 2) * np.cos(PH), np.sqrt(1 - MU ** 2) * np.sin(PH), MU], -1).reshape(-1, 3)
    w = (wmu[:, None] * np.full(48, np.pi / 24)[None, :]).reshape(-1)
    out = {"mesh": "icosphere4", "gap_edge": gap, "tol": 1e-8}
    for ka in (1.0, 1e-4):
        op = rf.Operator(m, ka, power_start=torch.from_numpy(synth.complex_start(m.N, 11)).cuda())
        e = m.rhs_gap([gap], [1.0])
        op.solve(e, tol=1e-8, maxit=2000)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        j, st, info = op.solve(e, tol=1e-8, maxit=2000)
        torch.cuda.synchronize()
        row = {"solve_ms": (time.perf_counter() - t0) * 1e3, "iters": info[0]["iters"], "status": st,
               "rel_residual": info[0]["rel_residual"]}
        if ka >= 1e-2:
            _, s = op.far_field(j, d)
            p_in = float(np.conj(j[0, gap].item()).real)
            p_rad = float(np.sum(w * s.cpu().numpy()[0])) / (4 * np.pi)
            row.update({"input_power": p_in, "radiated_power": p_rad, "power_balance": p_rad / p_in - 1})
        out[f"ka={ka:g}"] = row
        op.close()
    m.close()
    return out


def uneven_batch(rf, torch, concurrent=True, budget_gb=64.0):
    """The seeded uneven batch (32 icospheres, cubes and ellipsoids, N from
    480 to 16 200; 8 wavenumbers from 1e-3 to 5; 4 plane waves each): per
    object one rfcmp_op_create_many over the sweep (assembly, projectors,
    power iterations), then 4-right-hand-side BF16x3 solves with refinement
    to 1e-6.  concurrent: the objects are taken in groups whose operators
    (complex64 blocks and their BF16x3 planes) fit in budget_gb of device
    memory, and each group's solves go through one rfcmp_batch_solve;
    otherwise one object at a time and one rfcmp_solve per wavenumber.
    Whole-batch wall time, right-hand sides solved per second, and the
    iteration counts (the top wavenumber sits next to interior resonances of
    these bodies)."""
    from synth import batch
    objs = batch.uneven_objects()
    ks = batch.sweep_wavenumbers()
    groups, cur, used = [], [], 0.0
    for o, obj in enumerate(objs):
        C = len(obj["tri"])
        N = C * 3 // 2
        gb = len(ks) * (N * N + C * C) * 16 / 1e9
        if cur and (not concurrent or used + gb > budget_gb):
            groups.append(cur)
            cur, used = [], 0.0
        cur.append(o)
        used += gb
    groups.append(cur)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters, t_setup, t_solve, bad = [], 0.0, 0.0, 0
    for g in groups:
        ta = time.perf_counter()
        meshes, ops, es, kidx = [], [], [], []
        for o in g:
            m = rf.Mesh(objs[o]["xyz"], objs[o]["tri"])
            meshes.append(m)
            start = torch.from_numpy(synth.complex_start(m.N, 11)).cuda()
            for q, op in enumerate(rf.Operator.create_many(m, ks, power_start=start, precision=1)):
                kh, pol = batch.sweep_waves(o, q)
                ops.append(op)
                es.append(op.rhs_planewave(kh, pol))
                kidx.append(q)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        if concurrent:
            infos = rf.batch_solve(ops, es, tol=1e-6, maxit=4000)[2]
        else:
            infos = [op.solve(e, tol=1e-6, maxit=4000)[2] for op, e in zip(ops, es)]
        torch.cuda.synchronize()
        t_setup += tb - ta
        t_solve += time.perf_counter() - tb
        for q, info in zip(kidx, infos):
            bad += any(not i["rel_residual"] <= 1e-6 for i in info)
            iters.append((q, max(i["iters"] for i in info)))
        del es
        for op in ops:
            op.close()
        for m in meshes:
            m.close()
        rf.release_cached_memory()
    wall = time.perf_counter() - t0
    nrhs = len(objs) * len(ks) * 4
    low = [i for q, i in iters if q < len(ks) - 1]
    top = [i for q, i in iters if q == len(ks) - 1]
    return {"objects": len(objs), "wavenumbers": len(ks), "rhs": nrhs,
            "solver": "rfcmp_batch_solve" if concurrent else "rfcmp_solve", "groups": len(groups),
            "wall_s": wall, "setup_s": t_setup, "solve_s": t_solve, "rhs_per_s": nrhs / wall,
            "not_converged": int(bad),
            "iters_below_top_k": {"median": float(np.median(low)), "max": int(max(low))},
            "iters_top_k": {"median": float(np.median(top)), "max": int(max(top))}}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): this build has no multi-GPU path; "
              "one operator would shard by row blocks of T_A, V and L^+ with one all-gather of the input per "
              "product.", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    import torch
    import paper_1803_08333_amd as rf

    torch.cuda.init()
    dev = torch.device("cuda:0")
    xyz, tri = synth.icosphere(4)
    kh, pol = synth.default_plane_wave()
    N = len(tri) * 3 // 2
    C = len(tri)
    start = torch.from_numpy(synth.complex_start(N, 11)).to(dev)
    out = {}

    def step(record, **opts):
        m = rf.Mesh(xyz, tri)
        ops = rf.Operator.create_many(m, KS, power_start=start, **opts)
        es = [op.rhs_planewave(kh, pol) for op in ops]
        _, _, infos = rf.batch_solve(ops, es, tol=TOL, maxit=2000)
        for k, op, info in zip(KS, ops, infos):
            st = 0 if info[0]["rel_residual"] <= TOL else 1
            if record:
                a, b, g, lam = op.scalings()
                out[k] = {"status": st, "iters": info[0]["iters"], "restarts": info[0]["restarts"],
                          "rel_residual": info[0]["rel_residual"], "solve_ms": info[0]["ms_solve"],
                          "alpha": a, "beta": b, "gamma": g}
            op.close()
        m.close()

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()

    # one untimed step with every kernel tag timed: the per-kernel breakdown
    # and the choice of the dominant kernel
    base = ["cmatvec_ta", "cmatvec_v", "dmatvec_lp", "dmatvec_gll", "cmatvec_ta+v", "dmatvec_lp+gll"]
    tags = ["far_pairs", "near_pairs", "gather_ta"] + base + [f"{t}_nr{r}" for t in base for r in (2, 3, 4)] + \
        ["symv_reduce", "spd_inverse"]
    rf.profile_select(None)
    rf.profile_enable(True)
    step(False)
    torch.cuda.synchronize()
    brk = {t: rf.profile_read(t) for t in tags}
    rf.profile_enable(False)
    asm_ms = sum(brk[t][0] for t in ("far_pairs", "near_pairs", "gather_ta")) / len(KS)
    pairs_per_s = C * C / (asm_ms / 1e3)

    # roofline of the dominant kernel (largest total time)
    # symmetric products: the algorithmic bytes are the n (n + 1) / 2 distinct
    # entries (8 B each) plus x read and y written (16 B each, complex128) per
    # right-hand side; tags "<name>_nr<k>" are k right-hand sides per launch,
    # "<a>+<b>" two products sharing one launch
    def model(tag, avg_ms):
        name, nr = tag, 1
        if "_nr" in tag:
            name, nr = tag.split("_nr")[0], int(tag.split("_nr")[1])
        sizes = {"cmatvec_ta": [N], "cmatvec_v": [C], "dmatvec_lp": [C], "dmatvec_gll": [len(xyz)],
                 "cmatvec_ta+v": [N, C], "dmatvec_lp+gll": [C, len(xyz)]}.get(name)
        if sizes is not None:
            # the two-column T_A + V launches are the power iteration's, whose
            # V product takes one column
            nrs = [nr, 1 if (name == "cmatvec_ta+v" and nr == 2) else nr]
            byt = sum(8.0 * n * (n + 1) / 2 + 32.0 * n * nrs[q] for q, n in enumerate(sizes))
            return {"bound": "hbm", "achieved": byt / (avg_ms * 1e-3) / 1e9, "peak": HBM_GBS, "unit": "GB/s",
                    "algorithmic_bytes": byt}
        if tag == "far_pairs":
            fl = C * (C - 1) / 2 * 49 * FAR_FLOPS_PER_POINT_PAIR
            return {"bound": "alu", "achieved": fl / (avg_ms * 1e-3) / 1e12, "peak": FP32_VALU_TFLOPS,
                    "unit": "TFLOP/s"}
        return None

    ranked = sorted((v[0], t) for t, v in brk.items() if v[1] > 0 and model(t, 1.0) is not None)
    dom = ranked[-1][1]

    # timed steps: HIP events only around the dominant kernel's launches
    rf.profile_select([dom])
    rf.profile_enable(True)
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(i == args.steps - 1)
        print(f"# step {i + 1}/{args.steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = {dom: rf.profile_read(dom)}
    rf.profile_enable(False)
    rf.profile_select(None)
    ms_step = (t1 - t0) * 1e3 / args.steps
    value = len(KS) / (ms_step / 1e3)

    avg = prof[dom][0] / prof[dom][1]
    roof = model(dom, avg)
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = measured_traffic(dom)
    if roof["traffic"] is not None and "algorithmic_bytes" in roof:
        roof["traffic_over_algorithmic"] = roof["traffic"] / roof["algorithmic_bytes"]
    roof["kernel"] = dom
    roof["avg_ms"] = avg
    roof["launches"] = prof[dom][1]
    # The two wavenumbers' power iterations run on concurrent streams, so in
    # the timed steps a launch of the dominant kernel may share HBM with one
    # of the other wavenumber's.  The same step with them one after another
    # (streams = 1, untimed) gives the kernel alone on the device.
    rf.profile_select([dom])
    rf.profile_enable(True)
    step(False, streams=1)
    torch.cuda.synchronize()
    iso = rf.profile_read(dom)
    rf.profile_enable(False)
    rf.profile_select(None)
    iso_roof = model(dom, iso[0] / iso[1])
    roof["isolated"] = {"avg_ms": iso[0] / iso[1], "achieved": iso_roof["achieved"],
                        "frac": iso_roof["achieved"] / iso_roof["peak"], "launches": iso[1],
                        "note": "one untimed step with the power iterations one after another (streams = 1)"}

    res = {
        "metric": "RF-CMP solve time + EFIE assembly pairs/s; BF16x3 vs FP32 at 1e-6 residual",
        "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64 blocks (FP32 far-pair quadrature, FP64 near pairs), FP64 accumulation and projectors",
        "data": "synthetic (seeded icosphere, analytic plane wave)",
        "config": WORKLOAD,
        "solve_ms": {str(k): out[k]["solve_ms"] for k in KS},
        "iterations": {str(k): out[k]["iters"] for k in KS},
        "rel_residual": {str(k): out[k]["rel_residual"] for k in KS},
        "scalings": {str(k): [out[k]["alpha"], out[k]["beta"], out[k]["gamma"]] for k in KS},
        "assembly_pairs_per_s": pairs_per_s,
        "assembly_ms": asm_ms,
        "kernel_ms_per_step": {t: brk[t][0] for t in tags if brk[t][1] > 0},
        "bf16x3_vs_fp32": None,
        "spectral_study": None,
        "far_field": None,
        "roofline": roof,
    }
    if not args.no_precision_study:
        res["bf16x3_vs_fp32"] = precision_study(rf, torch, args.batch_rhs)
    if not args.no_spectral_study:
        res["spectral_study"] = spectral_study(rf)
        res["far_field"] = far_field_measurement(rf, torch)
        res["voltage_gap"] = voltage_gap_measurement(rf, torch)
    if args.uneven_batch:
        res["uneven_batch"] = uneven_batch(rf, torch)
        res["uneven_batch_serial"] = uneven_batch(rf, torch, concurrent=False)
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(xyz, tri, args.cpu_slab)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
