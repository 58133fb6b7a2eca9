"""Benchmark: RF-CMP EFIE solves on one MI355X.

Headline workload (the largest single-GPU configuration of the benchmark
set): PEC sphere r = 1 m, icosphere level 5 (C = 20480 cells, N = 30720 RWG),
ka = 2.0, 64 seeded plane waves (uniform directions, random polarisation),
BF16x3 operator products on MFMA with FP64-residual refinement to a true
relative residual of 1e-6.  One step = one pass of the whole hot path over it:
topology, projector set-up, far/near-pair assembly of T_A and V,
power-iteration scalings, the 64 excitations, preconditioned right-hand
sides, block CG with refinement, and recovery j = P_o i.  ``value`` =
right-hand sides solved per second over the timed steps.

Also reported (sub-keys): the level-4 sphere at ka = 1 and 1e-4 with one wave
each on the complex64/FP64 path (the former headline), the icosphere-2 case
solved by the FP64 oracle in full beside the GPU (error per result), the
precision study (BF16x3 against complex64/FP64 at equal residual), the
spectral study, far field, voltage gap, the compressed operator (ACA) at
icosphere levels 5-7, the uneven batch, and the oracle's CPU baseline.  Kernel durations come from HIP events the library records on
the launch stream.

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
FP64_MFMA_TFLOPS = 78.6

HEADLINE = {"workload": "PEC sphere r=1 m, icosphere level 5 (20480 cells, 30720 RWG), ka=2.0, 64 seeded plane "
                        "waves (uniform directions, random polarisation), BF16x3 products with FP64-residual "
                        "refinement to relative residual 1e-6",
            "mesh": "icosphere5", "ka": [2.0], "nrhs": 64, "precision": "bf16x3+fp64 refinement", "tol": 1e-6}
SWEEP = {"workload": "PEC sphere r=1 m, icosphere level 4 (5120 cells, 7680 RWG), ka=1.0 and ka=1e-4, "
                     "x-polarised plane wave along +z, complex64/FP64 path, CG to relative residual 1e-6",
         "mesh": "icosphere4", "ka": [1.0, 1e-4], "nrhs": 1, "precision": "c64 blocks, fp64 projectors", "tol": 1e-6}
TOL = 1e-6
FAR_FLOPS_PER_POINT_PAIR = 30     # sub 3, R^2 5, rsqrt 1, R 1, kR 1, sin+cos 2, G 3, moment sums 14 (FMA = 2)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-slab", type=int, default=64, help="1/slab of the test cells for the oracle sample")
    p.add_argument("--no-oracle-case", action="store_true")
    p.add_argument("--no-precision-study", action="store_true")
    p.add_argument("--no-spectral-study", action="store_true")
    p.add_argument("--batch-rhs", type=int, default=64)
    p.add_argument("--no-uneven-batch", action="store_true",
                   help="skip the uneven batch (32 objects x 8 wavenumbers x 4 plane waves, BF16x3)")
    p.add_argument("--no-compressed-study", action="store_true",
                   help="skip the compressed operator (ACA) at icosphere levels 5-7")
    p.add_argument("--compressed-only", type=int, nargs="+", default=None, metavar="LEVEL",
                   help="only the compressed-operator study, at these icosphere levels (8 waves each)")
    p.add_argument("--uneven-batch-serial", action="store_true",
                   help="also time the uneven batch with one rfcmp_solve per operator")
    p.add_argument("--copy-calibration", action="store_true",
                   help="only run a 1 GiB device copy (byte-counter calibration) and exit")
    return p.parse_args()


_BASELINE_MESH = {}


def _oracle_rows(args):
    """Rows of V and the cell-pair blocks for a set of test cells by the
    oracle's own sampled-row assembly (worker of cpu_baseline; the mesh is
    inherited from the parent process by fork)."""
    k, rows = args
    from threadpoolctl import threadpool_limits
    from oracle import assembly
    with threadpool_limits(limits=1):
        assembly.block_rows(_BASELINE_MESH["top"], k, rows)
    return len(rows)


def cpu_baseline(slab, head):
    """The FP64 oracle on the host cores, on a bounded sample of the headline
    workload (icosphere level 5, ka = 2, 64 plane waves), as it stands:
    * assembly: its sampled-row assembly (far-pair quadrature and near-pair
      integrals, the same functions as its full assembly) for every slab-th
      test cell, in groups of 8 rows over one process per core;
    * set-up and solve: its dense preconditioner (projectors, inverses), power
      scalings and CG on the same kind of problem at icosphere level 2
      (N = 480) with 64 plane waves, scaled to level 5 by N^3 (dense
      set-up) and N^2 (scalings and solve: dense products);
    solves/s = 64 / (full assembly + scaled set-up + scaled solve)."""
    import concurrent.futures
    from threadpoolctl import threadpool_info
    from oracle import assembly, rfcmp, rhs
    from oracle.topology import Topology
    k = HEADLINE["ka"][0]
    nrhs = HEADLINE["nrhs"]
    cores = min(os.cpu_count() or 1, 16)
    xyz, tri = synth.icosphere(5)
    top = Topology(xyz, tri)
    C = top.C
    rows = np.arange(0, C, slab)
    t0 = time.perf_counter()
    work = [(k, rows[i:i + 8]) for i in range(0, len(rows), 8)]
    _BASELINE_MESH["top"] = top
    import multiprocessing
    with concurrent.futures.ProcessPoolExecutor(max_workers=cores,
                                                mp_context=multiprocessing.get_context("fork")) as ex:
        list(ex.map(_oracle_rows, work))
    _BASELINE_MESH.clear()
    t_asm = time.perf_counter() - t0
    pairs_per_s = len(rows) * C / t_asm
    asm_full = C * C / pairs_per_s
    # dense set-up and solve at level 2
    x3, t3 = synth.icosphere(2)
    top3 = Topology(x3, t3)
    TA3, V3 = assembly.assemble(top3, k)
    t1 = time.perf_counter()
    pre = rfcmp.Preconditioner(top3, TA3, V3, k)
    t_setup = time.perf_counter() - t1
    t1 = time.perf_counter()
    pre.power_scalings(synth.complex_start(top3.N, 11), 30, tol=1e-2)
    kh, pol = synth.plane_waves(nrhs, 4)
    e = rhs.planewave(top3, k, kh, pol)
    b = pre.rhs(e.T)
    _, its, _ = rfcmp.cg(pre.apply, b, TOL, 1000)
    t_solve = time.perf_counter() - t1
    scale = top.N / top3.N
    total = asm_full + t_setup * scale ** 3 + t_solve * scale ** 2
    threads = max((x.get("num_threads", 1) for x in threadpool_info()), default=1)
    return {"value": nrhs / total, "unit": "solves/s", "cores": cores, "kind": "oracle", "cpu": cpu_model(),
            "sample": f"oracle sampled-row assembly of 1/{slab} of the level-5 test cells ({len(rows)} x {C} cell "
                      f"pairs, ka={k}) over {cores} processes in {t_asm:.1f} s, scaled to all C^2 pairs "
                      f"({asm_full:.0f} s); dense set-up ({t_setup:.1f} s) and power scalings + block CG on 64 "
                      f"waves ({t_solve:.1f} s, {its} iterations) at icosphere level 2 on {threads} BLAS "
                      f"threads, scaled by N^3 and N^2 to level 5; solves/s = 64 / total",
            "assembly_pairs_per_s": pairs_per_s, "phases_s": {"assembly": asm_full,
                                                             "setup": t_setup * scale ** 3,
                                                             "scalings_and_solve": t_solve * scale ** 2},
            "gpu_over_cpu": head["value"] / (nrhs / total)}


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

# HBM bytes per launch from two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE,
# KiB per dispatch, mean over the dispatches of the tag's kernel and grid),
# each scaled by what the same counter reads for a plain 1 GiB device copy
# (FETCH_SIZE reads 2^19 KiB for 2^30 bytes fetched: scale 2.0; WRITE_SIZE
# reads 2^20 KiB: scale 1.0), per workload and tag.  Valid only for the
# kernel source they were taken on: reported as null once that file changes.
TRAFFIC_SCALE = {"fetch": 2.0, "write": 1.0}
TRAFFIC = {
    "icosphere5_64rhs": {
        "gemm_ta": {"source": "paper_1803_08333_amd/csrc/gemm.hip",
                    "sha256": "3a9a7ba3393dd629b05455a8cc041999b61ce68e136862d80d6a7ab277421e29",
                    "kib": (3757129.2, 30720.0)},
        "zgemm_ta_nr32": {"source": "paper_1803_08333_amd/csrc/zgemm.hip",
                          "sha256": "6c2552a624e26ee57abf050493d1670743d56309a031422a97aaa2522169ef24",
                          "kib": (3979426.9, 122880.0)},
    },
}


def measured_traffic(tag, workload):
    import hashlib
    t = TRAFFIC.get(workload, {}).get(tag)
    if t is None:
        return None
    src = os.path.join(os.path.dirname(os.path.abspath(__file__)), t["source"])
    with open(src, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != t["sha256"]:
            return None
    fk, wk = t["kib"]
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
    paper's sphere study) on icosphere levels 1-5 and the jittered torus at
    48 x 24, 96 x 48 and 144 x 72 (N = 3456 to 31104): the
    CG-Lanczos estimate of a solve of A i = b with a seeded generic b (the
    library's rfcmp_solve_system), power-iteration scalings."""
    from paper_1803_08333_amd import study
    ks = [1.0, 1e-2, 1e-4, 1e-12, study.K_1E_25_HZ]
    meshes = {f"icosphere{L}": synth.icosphere(L) for L in (1, 2, 3, 4, 5)}
    # the genus-1 body refined twice (Fig. CubeTorus's 1/h axis)
    for nmaj, nmin in ((48, 24), (96, 48), (144, 72)):
        meshes[f"torus{nmaj}x{nmin}"] = synth.torus(nmaj, nmin)
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
    # the twelfth edge in lexicographic order of its vertex pair
    ev, _, _ = m.edges()
    gap = int(np.lexsort((ev.max(axis=1), ev.min(axis=1)))[11])
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
    to 1e-6, each over a shared block Krylov space (options.block_cg = 1; the
    default takes it from 8 right-hand sides on: with 4 it cuts the median
    iterations at the near-resonant top wavenumber from about 390 to 240).  concurrent: the objects are taken in groups whose operators
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
            for q, op in enumerate(rf.Operator.create_many(m, ks, power_start=start, precision=1, block_cg=1)):
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


def compressed_study(rf, torch, levels=((5, 8), (6, 8), (7, 8))):
    """The compressed operator (options.aca_tol = 1e-4: T_A and V as
    hierarchical matrices with ACA low-rank blocks, the compression of the
    paper's large example, Sec. 4) on icospheres at levels 5 (N = 30 720),
    6 (122 880) and 7 (491 520, whose dense blocks would take 2.8 TB), ka = 2,
    complex64 storage with FP64 accumulation: set-up time (mesh, tree, dense
    tiles, ACA, projector factors, power iteration), storage against the
    dense blocks, ranks, one block solve of seeded plane waves to 1e-6, and
    the roofline of the compressed T_A product in that solve (algorithmic
    bytes: the stored entries read once plus x in and y out)."""
    out = {"aca_tol": 1e-4, "ka": 2.0}
    for lvl, nw in levels:
        xyz, tri = synth.icosphere(lvl)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        m = rf.Mesh(xyz, tri)
        start = torch.from_numpy(synth.complex_start(m.N, 11)).cuda()
        rf.profile_select(None)
        rf.profile_enable(True)
        op = rf.Operator(m, 2.0, power_start=start, aca_tol=1e-4)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        setup = {t: rf.profile_read(t)[0] for t in ("hm_dense", "near_pairs", "hm_aca_ta", "hm_aca_v")}
        rf.profile_enable(False)
        info = op.compression()
        kh, pol = synth.plane_waves(nw, 4)
        e = op.rhs_planewave(kh, pol)
        rf.profile_enable(True)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        j, st, inf = op.solve(e, tol=1e-6, maxit=500)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        tot, nl = rf.profile_read(f"hm_matvec_ta_nr{nw}")
        totv, nlv = rf.profile_read(f"hm_matvec_v_nr{nw}")
        rf.profile_enable(False)
        N, C = m.N, m.C
        stored = [8.0 * (info["dense_entries"][q] + info["lowrank_entries"][q]) for q in (0, 1)]
        dense = [8.0 * N * N, 8.0 * C * C]
        prod = None
        if nl:
            avg = tot / nl
            byt = stored[0] + 32.0 * N * nw
            prod = {"launches": nl, "avg_ms": avg, "bound": "hbm", "algorithmic_bytes": byt,
                    "achieved": byt / (avg * 1e-3) / 1e9, "peak": HBM_GBS, "unit": "GB/s",
                    "frac": byt / (avg * 1e-3) / 1e9 / HBM_GBS, "v_avg_ms": totv / nlv if nlv else None}
        out[f"icosphere{lvl}"] = {
            "N": N, "C": C, "waves": nw, "setup_s": t1 - t0, "setup_kernels_ms": setup,
            "stored_gb": [x / 1e9 for x in stored], "dense_gb": [x / 1e9 for x in dense],
            "stored_over_dense": sum(stored) / sum(dense), "lowrank_blocks": info["lowrank_blocks"],
            "max_rank": info["max_rank"], "mean_rank": info["mean_rank"],
            "solve_ms": (t3 - t2) * 1e3, "status": st, "max_iters": max(i["iters"] for i in inf),
            "max_rel_residual": max(i["rel_residual"] for i in inf), "solves_per_s": nw / (t3 - t2),
            "product_ta": prod}
        print(f"# compressed operator, level {lvl} done", file=sys.stderr, flush=True)
        op.close()
        m.close()
        del e, j, start
        rf.release_cached_memory()
    return out


# ------------------------------------------------------------------ kernel models
# Algorithmic work per launch of each timed tag (what the method must do,
# not what the kernel happens to move):
#   symmetric products (cmatvec_*, dmatvec_*): the n (n + 1)/2 distinct
#     entries (8 B each: complex64 or FP64) plus x read and y written (16 B
#     each, complex128) per right-hand side; "<a>+<b>" = two products in one
#     launch, "_nr<k>" = k right-hand sides;
#   assemble_ta: C (C - 1)/2 unordered cell pairs x 49 point pairs x 30 flops
#     (the cell pairs each tile pair forms again for its own edges are
#     overhead, not algorithmic work);
#   gemm_<m>: BF16x3 product, three bf16 MFMA products per real multiply-add,
#     four real multiply-adds per complex one: 24 n^2 nr MFMA flops (complex
#     matrices), 6 n^2 (2 nr) for the real projector matrices;
#   spd_inverse: the symmetric Gauss-Jordan sweep reads and writes the upper
#     triangle once per 64-wide pivot block: (n/64) * 8 n^2 bytes.
FAR_FLOPS_PER_POINT_PAIR = 30     # sub 3, R^2 5, rsqrt 1, R 1, kR 1, sin+cos 2, G 3, moment sums 14 (FMA = 2)


def kernel_model(tag, avg_ms, sz, nrhs):
    """Roofline entry for one launch of `tag` (avg_ms per launch) on a mesh of
    sizes sz = {"N", "C", "V"}; None for tags without a model."""
    N, C, V = sz["N"], sz["C"], sz["V"]
    sec = avg_ms * 1e-3
    name, nr = tag, 1
    if "_nr" in tag:
        name, nr = tag.split("_nr")[0], int(tag.split("_nr")[1])
    sym = {"cmatvec_ta": [N], "cmatvec_v": [C], "dmatvec_lp": [C], "dmatvec_gll": [V],
           "cmatvec_ta+v": [N, C], "dmatvec_lp+gll": [C, V]}.get(name)
    if sym is not None:
        # the two-column T_A + V launches are the power iteration's, whose V
        # product takes one column
        nrs = [nr, 1 if (name == "cmatvec_ta+v" and nr == 2) else nr]
        byt = sum(8.0 * n * (n + 1) / 2 + 32.0 * n * nrs[q] for q, n in enumerate(sym))
        return {"bound": "hbm", "achieved": byt / sec / 1e9, "peak": HBM_GBS, "unit": "GB/s",
                "algorithmic_bytes": byt}
    if name == "assemble_ta":
        fl = C * (C - 1) / 2 * 49 * FAR_FLOPS_PER_POINT_PAIR
        return {"bound": "alu", "achieved": fl / sec / 1e12, "peak": FP32_VALU_TFLOPS, "unit": "TFLOP/s",
                "algorithmic_flops": fl}
    if name in ("zgemm_ta", "zgemm_v"):
        n = N if name == "zgemm_ta" else C
        fl = 8.0 * n * n * nr
        # the matrix cores execute three real products per complex one
        # (Gauss), over 16 or 32 columns
        mf = 6.0 * n * n * (16 if nr <= 16 else 32)
        byt = 8.0 * n * n + 32.0 * n * nr
        return {"bound": "mfma", "achieved": fl / sec / 1e12, "peak": FP64_MFMA_TFLOPS, "unit": "TFLOP/s",
                "algorithmic_flops": fl, "mfma_flops": mf, "mfma_tflops": mf / sec / 1e12,
                "algorithmic_bytes": byt, "matrix_bytes": 8.0 * n * n, "hbm_gbs": 8.0 * n * n / sec / 1e9,
                "floor_ms": {"hbm": byt / (HBM_GBS * 1e9) * 1e3, "mfma": fl / (FP64_MFMA_TFLOPS * 1e12) * 1e3}}
    if name.startswith("gemm_"):
        n = {"gemm_ta": N, "gemm_v": C, "gemm_lp": C, "gemm_gll": V, "gemm_gtp": C}.get(name)
        if n is None:
            return None
        fl = 24.0 * n * n * nrhs
        # the bound is the resource whose floor is the longer: the bf16 planes
        # (8 B per complex entry) plus x read and y written against HBM, or the
        # three-pass MFMA work against the bf16 peak
        byt = 8.0 * n * n + 32.0 * n * nrhs
        t_hbm, t_mfma = byt / (HBM_GBS * 1e9), fl / (BF16_MFMA_TFLOPS * 1e12)
        out = {"algorithmic_flops": fl / 3.0, "mfma_flops": fl, "mfma_tflops": fl / sec / 1e12,
               "mfma_frac": fl / sec / 1e12 / BF16_MFMA_TFLOPS, "algorithmic_bytes": byt,
               "matrix_bytes": 8.0 * n * n, "hbm_gbs": 8.0 * n * n / sec / 1e9,
               "floor_ms": {"hbm": t_hbm * 1e3, "mfma": t_mfma * 1e3}}
        if t_hbm >= t_mfma:
            out.update({"bound": "hbm", "achieved": byt / sec / 1e9, "peak": HBM_GBS, "unit": "GB/s"})
        else:
            out.update({"bound": "mfma", "achieved": fl / sec / 1e12, "peak": BF16_MFMA_TFLOPS, "unit": "TFLOP/s"})
        return out
    if name == "spd_inverse":
        # one launch = one inverse; the L^+ inverse (n = C) is the larger
        byt = (C / 64.0) * 8.0 * C * C
        return {"bound": "hbm", "achieved": byt / sec / 1e9, "peak": HBM_GBS, "unit": "GB/s",
                "algorithmic_bytes": byt, "note": "per launch as if every launch were the L^+ inverse (n = C); "
                                                 "the G_ll^-1 inverse (n = V) is smaller"}
    return None


ALL_TAGS_BASE = ["cmatvec_ta", "cmatvec_v", "dmatvec_lp", "dmatvec_gll", "cmatvec_ta+v", "dmatvec_lp+gll"]
SP_TAGS_BASE = ["spsolve_lp", "spsolve_gll", "spsolve_gtp", "spsolve_lp+gll", "spsolve_lp+gtp"]
ALL_TAGS = (["assemble_ta", "near_pairs"] + ALL_TAGS_BASE +
            [f"zgemm_{m}_nr{r}" for m in ("ta", "v") for r in range(1, 33)] +
            [f"{t}_nr{r}" for t in ALL_TAGS_BASE for r in (2, 3, 4)] +
            ["symv_reduce", "spd_inverse", "gemm_ta", "gemm_v", "gemm_lp", "gemm_gll", "gemm_gtp"] +
            SP_TAGS_BASE + [f"{t}_nr{r}" for t in SP_TAGS_BASE for r in list(range(2, 9)) + [16, 32, 64]])


def run_workload(rf, torch, wl, steps, warmup, label):
    """Time `steps` whole-path steps of one workload.  Returns the result
    dict: value (right-hand sides solved per second), ms_per_step, per-k
    reports, the per-kernel breakdown of one untimed profiled step, and the
    roofline of the dominant kernel (largest total time) measured with HIP
    events over the timed steps."""
    xyz, tri = wl["mesh_fn"]()
    ks = wl["ka"]
    nrhs = wl["nrhs"]
    prec = wl["precision_opt"]
    N = len(tri) * 3 // 2
    sz = {"N": N, "C": len(tri), "V": len(xyz)}
    if nrhs == 1:
        kh, pol = synth.default_plane_wave()
    else:
        kh, pol = synth.plane_waves(nrhs, wl["wave_seed"])
    start = torch.from_numpy(synth.complex_start(N, 11)).cuda()
    rec = {}

    def step(record, **opts):
        m = rf.Mesh(xyz, tri)
        ops = rf.Operator.create_many(m, ks, power_start=start, precision=prec, **opts)
        es = [op.rhs_planewave(kh, pol) for op in ops]
        _, st, infos = rf.batch_solve(ops, es, tol=TOL, maxit=2000)
        for k, op, info in zip(ks, ops, infos):
            if record:
                a, b, g, lam = op.scalings()
                rec[k] = {"status": st, "max_iters": max(i["iters"] for i in info),
                          "max_restarts": max(i["restarts"] for i in info),
                          "max_rel_residual": max(i["rel_residual"] for i in info),
                          "converged": all(i["rel_residual"] <= TOL for i in info),
                          "solve_ms": info[0]["ms_solve"], "power_steps": op.power_steps(),
                          "alpha": a, "beta": b, "gamma": g}
            op.close()
        m.close()
        if st != 0:
            raise RuntimeError(f"{label}: rfcmp_batch_solve returned status {st}")

    for _ in range(warmup):
        step(False)
    torch.cuda.synchronize()
    print(f"# {label}: warmup done", file=sys.stderr, flush=True)

    # one untimed step with every kernel tag timed: the breakdown and the
    # choice of the dominant kernel (largest total time among all tags)
    rf.profile_select(None)
    rf.profile_enable(True)
    step(False)
    torch.cuda.synchronize()
    brk = {t: rf.profile_read(t) for t in ALL_TAGS}
    rf.profile_enable(False)
    brk = {t: v for t, v in brk.items() if v[1] > 0}
    ranked = sorted(brk.items(), key=lambda kv: -kv[1][0])
    dom = ranked[0][0]
    asm_ms = sum(brk.get(t, (0.0, 0))[0] for t in ("assemble_ta", "near_pairs")) / len(ks)

    # timed steps: HIP events only around the dominant kernel's launches
    rf.profile_select([dom])
    rf.profile_enable(True)
    t0 = time.perf_counter()
    for i in range(steps):
        step(i == steps - 1)
        print(f"# {label}: step {i + 1}/{steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dtot, dn = rf.profile_read(dom)
    rf.profile_enable(False)
    rf.profile_select(None)
    ms_step = (t1 - t0) * 1e3 / steps
    avg = dtot / dn
    roof = kernel_model(dom, avg, sz, nrhs) or {"bound": None, "achieved": None, "peak": None, "unit": None}
    if roof.get("achieved") is not None:
        roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = measured_traffic(dom, wl["name"])
    if roof["traffic"] is not None and roof.get("algorithmic_bytes"):
        roof["traffic_over_algorithmic"] = roof["traffic"] / roof["algorithmic_bytes"]
    roof.update({"kernel": dom, "avg_ms": avg, "launches": dn, "launches_per_step": dn / steps})
    kernels = {}
    for t, (tot, n) in ranked:
        e = {"ms_per_step": tot, "launches": n, "avg_ms": tot / n}
        mdl = kernel_model(t, tot / n, sz, nrhs)
        if mdl is not None:
            e.update({"bound": mdl["bound"], "achieved": mdl["achieved"], "unit": mdl["unit"],
                      "frac": mdl["achieved"] / mdl["peak"]})
        kernels[t] = e
    return {"value": len(ks) * nrhs / (ms_step / 1e3), "ms_per_step": ms_step, "per_k": {str(k): rec[k] for k in ks},
            "assembly_ms_per_k": asm_ms, "assembly_pairs_per_s": sz["C"] ** 2 / (asm_ms / 1e3),
            "kernels": kernels, "roofline": roof, "dominant": dom}


WORKLOADS = {
    "icosphere5_64rhs": dict(HEADLINE, name="icosphere5_64rhs", mesh_fn=lambda: synth.icosphere(5),
                             precision_opt=1, wave_seed=4),
    "icosphere4_two_k": dict(SWEEP, name="icosphere4_two_k", mesh_fn=lambda: synth.icosphere(4),
                             precision_opt=0, wave_seed=None),
}


def oracle_case(rf, torch):
    """The icosphere-2 case (N = 480, ka = 0.1, one x-polarised wave along
    +z, CG to 1e-8) run in full by the FP64 oracle on the host (assembly,
    projectors, power scalings, CG) and by the GPU on both precision paths:
    wall time of each phase of the oracle, the GPU solve time, and the error
    of each GPU result against the oracle's j (whole, loop part, star part)."""
    from threadpoolctl import threadpool_info
    from oracle import assembly, rfcmp, rhs
    from oracle.topology import Topology
    k, tol = 0.1, 1e-8
    xyz, tri = synth.icosphere(2)
    kh, pol = synth.default_plane_wave()
    ph = {}
    t = time.perf_counter()
    top = Topology(xyz, tri)
    ph["topology_s"] = time.perf_counter() - t
    t = time.perf_counter()
    TA, V = assembly.assemble(top, k)
    ph["assembly_s"] = time.perf_counter() - t
    t = time.perf_counter()
    pre = rfcmp.Preconditioner(top, TA, V, k)
    ph["projectors_s"] = time.perf_counter() - t
    t = time.perf_counter()
    pre.power_scalings(synth.complex_start(top.N, 11), 30, tol=1e-2)
    ph["scalings_s"] = time.perf_counter() - t
    t = time.perf_counter()
    e = rhs.planewave(top, k, kh, pol)[0]
    b = pre.rhs(e)
    i, its, res = rfcmp.cg(pre.apply, b, tol, 1000)
    jref = pre.recover(i)
    ph["rhs_and_solve_s"] = time.perf_counter() - t
    ph["total_s"] = sum(ph.values())
    ph["cg_iters"] = its
    ph["blas_threads"] = max((x.get("num_threads", 1) for x in threadpool_info()), default=1)
    out = {"workload": "icosphere level 2 (320 cells, 480 RWG), ka=0.1, x-polarised wave along +z, CG to 1e-8",
           "oracle": ph}
    m = rf.Mesh(xyz, tri)
    start = torch.from_numpy(synth.complex_start(m.N, 11)).cuda()
    for prec in (0, 1):
        op = rf.Operator(m, k, power_start=start, precision=prec)
        eg = op.rhs_planewave(kh, pol)
        op.solve(eg, tol=tol, maxit=1000)
        torch.cuda.synchronize()
        t = time.perf_counter()
        j, st, info = op.solve(eg, tol=tol, maxit=1000)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) * 1e3
        jg = j.cpu().numpy()[0]
        rel = lambda a, r: float(np.linalg.norm(a - r) / np.linalg.norm(r))
        out["bf16x3" if prec else "fp32"] = {
            "solve_ms": ms, "iters": info[0]["iters"], "status": st, "rel_residual": info[0]["rel_residual"],
            "err_vs_oracle": rel(jg, jref), "err_loop_part": rel(pre.P_LH @ jg, pre.P_LH @ jref),
            "err_star_part": rel(pre.P_S @ jg, pre.P_S @ jref)}
        op.close()
    m.close()
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the library has no multi-GPU path; "
              "one operator would shard by row blocks of T_A, V and L^+ with one all-gather of the input per "
              "product.", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    import torch
    import paper_1803_08333_amd as rf

    torch.cuda.init()
    if args.compressed_only:
        print(json.dumps(compressed_study(rf, torch, levels=tuple((lv, 8) for lv in args.compressed_only))))
        return
    head = run_workload(rf, torch, WORKLOADS["icosphere5_64rhs"], args.steps, args.warmup, "icosphere5_64rhs")
    sweep = run_workload(rf, torch, WORKLOADS["icosphere4_two_k"], max(args.steps, 5), args.warmup,
                         "icosphere4_two_k")
    res = {
        "metric": "RF-CMP solve time + EFIE assembly pairs/s; BF16x3 vs FP32 at 1e-6 residual",
        "value": head["value"], "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16x3 MFMA products (FP32 accumulation) over c64 blocks, FP64 projectors and refinement "
                 "residual; FP32 far-pair quadrature, FP64 near pairs",
        "data": "synthetic (seeded icosphere, seeded plane waves)",
        "config": {k: v for k, v in HEADLINE.items()},
        "per_k": head["per_k"],
        "assembly_pairs_per_s": head["assembly_pairs_per_s"],
        "assembly_ms": head["assembly_ms_per_k"],
        "kernels": head["kernels"],
        "roofline": head["roofline"],
        "icosphere4_two_k": {"config": SWEEP, "value": sweep["value"], "unit": "solves/s",
                             "ms_per_step": sweep["ms_per_step"], "per_k": sweep["per_k"],
                             "assembly_pairs_per_s": sweep["assembly_pairs_per_s"],
                             "assembly_ms": sweep["assembly_ms_per_k"], "kernels": sweep["kernels"],
                             "roofline": sweep["roofline"]},
    }
    print("# headline and level-4 workloads done", file=sys.stderr, flush=True)
    if not args.no_precision_study:
        res["bf16x3_vs_fp32"] = precision_study(rf, torch, args.batch_rhs)
        print("# precision study done", file=sys.stderr, flush=True)
    if not args.no_spectral_study:
        res["spectral_study"] = spectral_study(rf)
        res["far_field"] = far_field_measurement(rf, torch)
        res["voltage_gap"] = voltage_gap_measurement(rf, torch)
        print("# spectral study, far field, voltage gap done", file=sys.stderr, flush=True)
    if not args.no_compressed_study:
        res["compressed_operator"] = compressed_study(rf, torch)
    if not args.no_uneven_batch:
        res["uneven_batch"] = uneven_batch(rf, torch)
        print("# uneven batch done", file=sys.stderr, flush=True)
    if args.uneven_batch_serial:
        res["uneven_batch_serial"] = uneven_batch(rf, torch, concurrent=False)
    if not args.no_cpu_baseline:
        # the CPU leg: the oracle timed on the host, and the GPU results of a
        # case it solves in full checked against it
        res["cpu_baseline"] = cpu_baseline(args.cpu_slab, head)
        if not args.no_oracle_case:
            res["cpu_baseline"]["oracle_case"] = oracle_case(rf, torch)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
