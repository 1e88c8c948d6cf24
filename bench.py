#!/usr/bin/env python3
"""Benchmark of the plane-wave H|psi> / Davidson path on one MI355X.

Workload (default): the 64-atom diamond-structure cell (a = 20.52 bohr, 30 Ry,
72^3 grid, 16 k-points of a shifted 4x4x1 mesh, 160 bands, 256 projectors),
synthetic seeded inputs already resident in HBM.  One step = one qm_apply_h
over every k-point and band (scatter, pruned inverse FFT, V(r), forward FFT,
gather + kinetic, projector GEMMs).  The JSON line reports bands/s, the
roofline of the dominant kernel (HIP events around each stage) and the FP64
CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0}
# vector ALU peak without packed-FP32 instructions (the kernels are built without them):
# 256 CUs x 2.4 GHz x 128 flop/clk (64 FMA lanes x 2) = 78.6 TFLOP/s for float32 and float64
ALU_PEAK_TFLOPS = 78.6
PREC_CODE = {"fp64": 0, "fp32": 1, "mixed": 2}
PREC_DTYPE = {"fp64": "f64", "fp32": "f32", "mixed": "f32+bf16"}


def _nsticks(miller, grid):
    i = np.mod(miller[:, :2], np.asarray(grid[:2]))
    return len(np.unique(i[:, 0] * grid[1] + i[:, 1]))


def _nax(miller, grid):
    return len(np.unique(np.mod(miller[:, 0], grid[0])))


def _fft_flops(n):
    return 5.0 * n * np.log2(n)


def build_inputs(w):
    import torch
    miller = np.concatenate(w.miller).astype(np.int32)
    beta = torch.empty(int(w.nproj * w.npw.sum()), dtype=torch.complex128, device="cuda")
    off = 0
    for ik in range(w.nk):
        b = torch.from_numpy(w.beta(ik).reshape(-1))
        beta[off:off + b.numel()].copy_(b)
        off += b.numel()
    vloc = torch.from_numpy(w.vloc_r()).cuda()
    psi = torch.empty(int(w.nbnd * w.npw.sum()), dtype=torch.complex128, device="cuda")
    off = 0
    for ik in range(w.nk):
        p = torch.from_numpy(w.psi(ik).reshape(-1))
        psi[off:off + p.numel()].copy_(p)
        off += p.numel()
    return miller, beta, vloc, psi


def algorithmic_model(w, prec):
    """Per-band minimal HBM bytes of each local stage and flops of the projector GEMMs."""
    csz = 16 if prec == "fp64" else 8
    out = {}
    nst = [_nsticks(m, w.grid) for m in w.miller]
    n3 = w.grid[2]
    tot_bands = w.nk * w.nbnd
    sb = sum(w.nbnd * s * n3 * csz for s in nst)          # stick buffer, all bands
    psi_b = sum(w.nbnd * int(n) * 16 for n in w.npw)      # c128 band block
    out["zinv"] = ("hbm", psi_b + sb)
    n1, n2 = w.grid[0], w.grid[1]
    xy_fl = 0.0
    for m in w.miller:
        nax = _nax(m, w.grid)
        xy_fl += w.nbnd * n3 * ((2 * nax + 2 * n2) * _fft_flops(n1) + 2.0 * n1 * n2)
    out["xy"] = ("alu", xy_fl)
    out["zfwd"] = ("hbm", sb + 2 * psi_b)
    fl = sum(8.0 * w.nproj * w.nbnd * int(n) for n in w.npw)
    out["proj_gemm"] = ("mfma", fl)
    out["expand_gemm"] = ("mfma", fl)
    return out, tot_bands, nst


# Files whose contents define the H|psi> kernels; the HBM traffic recorded from hardware
# counters is reported only while their hash matches the one stored with the counters.
KERNEL_SOURCES = ["cplx.h", "fft_kernels.h", "fft_launch.h", "fft_common.hip", "fft_f64.hip",
                  "fft_f32.hip", "gemm.hip", "nonlocal.hip", "plan.hip", "qm_internal.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hpsi_c3_hbm_traffic.txt")


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2308_07277_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(workload_name, prec, stage):
    """HBM bytes per launch of the stage's kernel from the committed FETCH_SIZE /
    WRITE_SIZE counter summary (each scaled by the copy calibration), or None."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    rec, meta = None, {}
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            if line.startswith("#") or "=" not in line:
                continue
            kv = dict(t.split("=", 1) for t in line.split())
            if "sources_sha256" in kv:
                meta = kv
            elif kv.get("workload") == workload_name and kv.get("prec") == prec and kv.get("stage") == stage:
                rec = kv
    if rec is None or meta.get("sources_sha256") != kernel_sources_sha256():
        return None
    return 1024.0 * (float(rec["fetch_kib"]) * float(meta["fetch_scale"]) +
                     float(rec["write_kib"]) * float(meta["write_scale"]))


def cpu_model():
    """The host CPU's model name (lscpu, else /proc/cpuinfo) and the cores this process may use."""
    name = None
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                name = line.split(":", 1)[1].strip()
    except Exception:
        pass
    if name is None and os.path.exists("/proc/cpuinfo"):
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                name = line.split(":", 1)[1].strip()
                break
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return name, cores


def cpu_baseline(w, nb_sample, nk_sample=8, threads=1):
    """The FP64 oracle on the first nk_sample k-points with nb_sample bands each, with the
    BLAS and FFT thread pools limited to `threads`."""
    from threadpoolctl import threadpool_limits
    import scipy.fft  # noqa: F401  (the oracle's FFT library is numpy.fft; scipy only counts threads)
    from oracle import hamiltonian as ham
    v = w.vloc_r()
    d = w.dmat()
    nk = min(nk_sample, w.nk)
    dt = 0.0
    with threadpool_limits(threads):
        for ik in range(nk):
            beta = w.beta(ik)
            psi = w.psi(ik)[:nb_sample]
            t0 = time.perf_counter()
            ham.apply_h_ref(w.cell, w.grid, w.k_cryst[ik], w.miller[ik], v, beta, d, psi)
            dt += time.perf_counter() - t0
    model, _ = cpu_model()
    return {"value": nk * nb_sample / dt, "unit": "bands/s", "cores": threads, "kind": "oracle",
            "cpu_model": model,
            "sample": f"apply_h_ref (numpy FFT + BLAS, float64, BLAS threads {threads}) on k-points "
                      f"0-{nk - 1} of the {w.name} workload, {nb_sample} bands each: {nk * nb_sample} "
                      f"band applications in {dt:.1f} s"}


def _plan_for(w, prec=0, nbnd_max=None):
    import paper_2308_07277_amd as qm
    miller, beta, vloc, _ = build_inputs(w)
    plan = qm.qm_hpsi_plan_create(w.cell, w.grid, w.k_cart, w.npw, miller,
                                  nbnd_max or w.nbnd, w.nproj, vloc, beta, w.dmat(), prec)
    return plan


def train_preconditioner(steps=1200, max_resid=1e-3):
    """Train the learned preconditioner on two 8-atom cells (all arithmetic on the GPU):
    the 25 Ry, 4 k, 32-band cell and the same cell at 30 Ry with 12 k and 20 bands.
    Rows come from Teter Davidson runs, late phase only (band residual <= max_resid);
    the residual-amplitude input is frozen at zero.  Returns (weights, info)."""
    import torch
    import workload
    from paper_2308_07277_amd import train as tr
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    parts = []
    for name in ("c2", "t2"):
        w = workload.make_workload(name)
        plan = _plan_for(w)
        psi = torch.cat([torch.from_numpy(w.psi(ik, purpose=2).reshape(-1)) for ik in range(w.nk)]).cuda()
        parts.append(tr.collect_pairs(plan, psi, w.nbnd, max_resid=max_resid))
        plan.close()
    data = tr.concat(parts[0], parts[1])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    weights, hist = tr.train(data, steps=steps)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    l_final = tr.full_loss(weights, data)
    l_init = tr.full_loss(tr.init_weights(0), data)
    return weights, {"cells": "8-atom cell: 25 Ry 4 k 32 bands, and 30 Ry 12 k 20 bands",
                     "rows": int(data["feat"].shape[0]), "bands": int(len(data["band_ptr"]) - 1),
                     "max_band_resid": max_resid, "frozen_inputs": [3],
                     "pair_gen_s": t1 - t0, "train_s": t2 - t1, "adam_steps": steps,
                     "loss_teter": l_init, "loss_final": l_final}


def hpsi_rates(name, steps=20, warmup=3):
    """H|psi> bands/s of one workload in each precision (all k, all bands per call)."""
    import torch
    import workload
    import paper_2308_07277_amd as qm
    w = workload.make_workload(name)
    miller, beta, vloc, psi = build_inputs(w)
    plan = qm.qm_hpsi_plan_create(w.cell, w.grid, w.k_cart, w.npw, miller, w.nbnd, w.nproj,
                                  vloc, beta, w.dmat(), 0)
    del beta, vloc
    hpsi = torch.empty_like(psi)
    qm.qm_hpsi_plan_autotune(plan, w.nbnd)
    out = {"grid": list(w.grid), "nk": w.nk, "nbnd": w.nbnd, "nproj": w.nproj,
           "npw": [int(w.npw.min()), int(w.npw.max())]}
    for prec in PREC_CODE:
        qm.qm_hpsi_plan_set_precision(plan, PREC_CODE[prec])
        for _ in range(warmup):
            qm.qm_apply_h(plan, -1, psi, hpsi, w.nbnd)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            qm.qm_apply_h(plan, -1, psi, hpsi, w.nbnd)
        torch.cuda.synchronize()
        ms_ = 1000.0 * (time.perf_counter() - t0) / steps
        out[prec] = {"bands_per_s": w.nk * w.nbnd / (ms_ / 1000.0), "ms_per_call": ms_}
    plan.close()
    return out


def davidson_cpu_baseline(name="c2", tol=1e-8):
    """The FP64 oracle Davidson (one thread) against the GPU solve from the same start on a
    cell the oracle finishes in seconds; returns times, iterations and eigenvalue agreement."""
    import torch
    from threadpoolctl import threadpool_limits
    import workload
    import paper_2308_07277_amd as qm
    from oracle import davidson as odav, hamiltonian as ham
    w = workload.make_workload(name)
    v = w.vloc_r()
    d = w.dmat()
    eig_cpu, its, t_cpu = [], [], 0.0
    with threadpool_limits(1):
        for ik in range(w.nk):
            m = w.miller[ik]
            beta = w.beta(ik)
            kin = ham.kinetic(w.cell, w.k_cryst[ik], m)
            h = lambda x, ik=ik, m=m, beta=beta: ham.apply_h_ref(w.cell, w.grid, w.k_cryst[ik], m, v,
                                                                 beta, d, x)
            t0 = time.perf_counter()
            r = odav.davidson_ref(h, w.psi(ik, purpose=2), kin, tol=tol)
            t_cpu += time.perf_counter() - t0
            eig_cpu.append(r["eig"])
            its.append(int(r["iterations"]))
    plan = _plan_for(w)
    start = torch.cat([torch.from_numpy(w.psi(ik, purpose=2).reshape(-1)) for ik in range(w.nk)]).cuda()
    psi = start.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    eig, res, stats, st = qm.qm_davidson_solve(plan, -1, psi, w.nbnd, tol=tol, max_iter=400)
    torch.cuda.synchronize()
    t_gpu = time.perf_counter() - t0
    plan.close()
    return {"workload": f"{name}: {len(w.atoms)} atoms, {w.nk} k, {w.nbnd} bands, tol {tol:g} Ha",
            "cpu_oracle_s": t_cpu, "cpu_cores": 1, "cpu_iterations": its, "gpu_s": t_gpu,
            "gpu_iterations": stats["iterations"], "gpu_status": int(st),
            "max_abs_eig_diff": float(np.abs(np.array(eig_cpu) - eig).max())}


# Davidson arms: (name, ladder precision of H or None for float64 throughout, switch
# residual, preconditioner, buffer bands: None = the run's default, lanes: None = default,
# subspace_fp32).  The ladder arms keep residual norms, Rayleigh-Ritz, CholQR and the
# projected eigenproblem in float64; the arms marked "f32 subspace" also run the subspace
# products in float32 arithmetic before the switch.
DAVIDSON_ARMS = [
    ("fp64+teter", None, 0.0, "teter", None, None, 0),
    ("fp64+teter, one lane", None, 0.0, "teter", None, 1, 0),
    ("fp64+teter, no buffer bands", None, 0.0, "teter", 0, None, 0),
    ("fp64+mlp", None, 0.0, "mlp", None, None, 0),
    ("fp32-ladder+teter", 1, 3e-4, "teter", None, None, 0),
    ("fp32-ladder+mlp", 1, 3e-4, "mlp", None, None, 0),
    ("bf16-ladder+teter", 2, 1e-3, "teter", None, None, 0),
    ("bf16-ladder+mlp", 2, 1e-3, "mlp", None, None, 0),
    ("fp32-ladder+mlp, f32 subspace", 1, 3e-4, "mlp", None, None, 1),
    ("bf16-ladder+mlp, f32 subspace", 2, 1e-3, "mlp", None, None, 1),
]
HEADLINE_ARMS = ("fp64+teter", "fp32-ladder+mlp")


def oracle_residuals(w, xs, eig, kpts, bands=None, threads=None):
    """||H x - theta x|| of returned Ritz pairs with H from oracle.hamiltonian (float64 CPU)."""
    from threadpoolctl import threadpool_limits
    from oracle import hamiltonian as ham
    v, d = w.vloc_r(), w.dmat()
    out = {}
    with threadpool_limits(threads):
        for ik in kpts:
            b = list(range(w.nbnd)) if bands is None else list(bands)
            x = xs[ik][b]
            hx = ham.apply_h_ref(w.cell, w.grid, w.k_cryst[ik], w.miller[ik], v, w.beta(ik), d, x)
            out[ik] = np.linalg.norm(hx - eig[ik][b, None] * x, axis=1)
    return out


def fp64_residuals(plan, w, psi, eig):
    """Largest ||H x - theta x|| per k-point, H applied by the library in float64."""
    import torch
    import paper_2308_07277_amd as qm
    hx = torch.empty_like(psi)
    qm.qm_apply_h(plan, -1, psi, hx, w.nbnd)
    out, off = [], 0
    for ik in range(w.nk):
        n = w.nbnd * int(w.npw[ik])
        x = psi[off:off + n].view(w.nbnd, -1)
        th = torch.from_numpy(np.ascontiguousarray(eig[ik])).to(psi.device)
        r = hx[off:off + n].view(w.nbnd, -1) - th[:, None] * x
        out.append(float(torch.linalg.vector_norm(r, dim=1).max()))
        off += n
    return np.array(out)


def _split_k(flat, w, nbnd):
    out, off = [], 0
    for ik in range(w.nk):
        n = nbnd * int(w.npw[ik])
        out.append(flat[off:off + n].reshape(nbnd, int(w.npw[ik])))
        off += n
    return out


def davidson_run(name, weights=None, tol=1e-8, max_basis_factor=4, lanes=3, only=None,
                 extra_bands=32, repeats=2, oracle_k=(0,), oracle_bands=None):
    """Block Davidson from a seeded random start to max residual <= tol over every k-point
    and wanted band, per arm of DAVIDSON_ARMS: float64 H, or a precision ladder (float32
    FFT with float32 or bf16 projector GEMMs while the max residual is above the switch
    residual, float64 H below), with the Teter or the learned preconditioner, and
    extra_bands buffer bands (corrected but not required to converge).

    Every arm first runs one untimed solve of a single iteration with its own band, basis
    and lane settings (workspace allocation and first launches), then `repeats` timed solves
    in alternating arm order; time_s is their median.  For the HEADLINE_ARMS the returned
    Ritz pairs are checked against the FP64 oracle: residuals ||H x - theta x|| with the
    oracle's H at the k-points oracle_k (bands oracle_bands, default all), and with the
    library's float64 H (parity-tested against the oracle to 1e-12) at every k-point.  Each
    residual bounds its eigenvalue's error against the exact eigenvalue (Krylov-Weinstein)."""
    import torch
    import workload
    import paper_2308_07277_amd as qm
    w = workload.make_workload(name)
    plan = _plan_for(w, prec=2, nbnd_max=w.nbnd + extra_bands)
    start = torch.cat([torch.from_numpy(w.psi(ik, purpose=2).reshape(-1)) for ik in range(w.nk)]).cuda()
    sel = [a for a in DAVIDSON_ARMS
           if (only is None or a[0] in only) and not (a[3] == "mlp" and weights is None)]

    def solve(arm, max_iter=400):
        _, lprec, sw, pre, eb, ln, s32 = arm
        eb = extra_bands if eb is None else eb
        kw = dict(precond=qm.QM_PRECOND_MLP if pre == "mlp" else qm.QM_PRECOND_TETER,
                  switch_resid=sw, lanes=lanes if ln is None else ln, extra_bands=eb,
                  max_basis=int(max_basis_factor * (w.nbnd + eb)), subspace_fp32=s32)
        if pre == "mlp":
            kw["mlp_weights"] = weights
        qm.qm_hpsi_plan_set_precision(plan, 0 if lprec is None else lprec)
        psi = start.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        eig, res, stats, st = qm.qm_davidson_solve(plan, -1, psi, w.nbnd, tol=tol, max_iter=max_iter, **kw)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, eig, res, stats, st, psi, eb

    arms, eigs, times = {}, {}, {a[0]: [] for a in sel}
    for rep in range(repeats):
        for arm in (sel if rep % 2 == 0 else sel[::-1]):
            if rep == 0:
                solve(arm, max_iter=1)       # untimed: this arm's workspace and first launches
            wall, eig, res, stats, st, psi, eb = solve(arm)
            times[arm[0]].append(wall)
            if rep == 0:
                eigs[arm[0]] = eig
                arms[arm[0]] = {"status": int(st), "iterations": stats["iterations"],
                                "n_hpsi_bands": stats["n_hpsi_bands"],
                                "n_hpsi_bands_lowp": stats["n_hpsi_bands_lowp"],
                                "max_resnorm": stats["max_resnorm"], "t_hpsi_ms": stats["t_hpsi_ms"],
                                "t_eig_ms": stats["t_eig_ms"], "t_subspace_ms": stats["t_subspace_ms"],
                                "gram_schmidt_calls": stats["n_gs"],
                                "gram_schmidt_second_passes": stats["n_gs_second"],
                                "extra_bands": eb, "switch_resid": arm[2],
                                "subspace": "float32 before the switch" if arm[6] else "float64"}
                if arm[0] in HEADLINE_ARMS and st == 0:
                    xs = _split_k(psi.cpu().numpy(), w, w.nbnd)
                    ro = oracle_residuals(w, xs, eig, oracle_k, oracle_bands)
                    qm.qm_hpsi_plan_set_precision(plan, 0)
                    rgn = fp64_residuals(plan, w, psi, eig)
                    arms[arm[0]]["eig_error_bound"] = {
                        "oracle_k": list(oracle_k),
                        "oracle_bands": "all" if oracle_bands is None else list(oracle_bands),
                        "oracle_resid_max": float(max(v.max() for v in ro.values())),
                        "oracle_resid_max_per_k": {int(k): float(v.max()) for k, v in ro.items()},
                        "fp64_h_resid_max_all_k": float(rgn.max()),
                        "fp64_h_resid_max_per_k": [float(v) for v in rgn]}
    for arm in arms:
        ts = sorted(times[arm])
        arms[arm]["time_s"] = float(np.median(ts))
        arms[arm]["time_s_runs"] = times[arm]
    ref = "fp64+teter" if "fp64+teter" in eigs else next(iter(eigs))
    for arm in arms:
        if arm != ref:
            arms[arm]["max_abs_eig_diff_vs_" + ref] = float(np.abs(eigs[arm] - eigs[ref]).max())
            if arms[arm]["status"] == 0 and arms[ref]["status"] == 0:
                arms[arm]["speedup_vs_" + ref] = arms[ref]["time_s"] / arms[arm]["time_s"]
    plan.close()
    return {"workload": f"{name}: {len(w.atoms)}-atom cell, {w.nk} k-points, "
                        f"{w.nbnd} bands, tol {tol:g} Ha, {extra_bands} buffer bands, max_basis "
                        f"{max_basis_factor} (nbnd + buffer bands), k-points in {lanes} concurrent "
                        f"lanes, unless the arm says otherwise; time_s is the median of {repeats} "
                        f"solves after an untimed one-iteration solve per arm",
            "arms": arms, "lowest_eig_gamma": float(eigs[ref][0][0]),
            "eig_error_bound_note": "eig_error_bound: residual norms of the returned Ritz pairs "
                                    "recomputed with the FP64 CPU oracle's H (oracle_k) and with the "
                                    "library's float64 H (all k); each bounds the error of its "
                                    "eigenvalue against the exact one (Krylov-Weinstein)"}


def _timed(fn, reps):
    """Median wall time (s) of fn() over reps calls, each bracketed by device synchronisation,
    after one untimed call."""
    import torch
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts))


def _cpu_timed(fn, reps=1):
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts))


def adjacent_rows(reps=5):
    """The parts built on the H|psi> kernels, each timed on the GPU (median of reps calls
    after an untimed one) with the FP64 CPU oracle timed beside it on a bounded sample:
    electron density and Hartree potential on the 64-atom cell, the Hartree-only SCF on the
    2- and 8-atom cells, ETRS real-time propagation and GW plane-wave matrix elements on the
    64-atom cell."""
    import torch
    import workload
    import paper_2308_07277_amd as qm
    from oracle import density as od, tddft as otd, gw as ogw, hamiltonian as ham
    out = {}
    w = workload.make_workload("c3")
    miller, beta, vloc, psi = build_inputs(w)
    plan = qm.qm_hpsi_plan_create(w.cell, w.grid, w.k_cart, w.npw, miller, w.nbnd, w.nproj,
                                  vloc, beta, w.dmat(), 0)
    nst = _nsticks(w.miller[0], w.grid)
    bands = w.nk * w.nbnd
    # density: sphere -> sticks -> planes, |psi(r)|^2 accumulated over every k and band
    rho = torch.empty(tuple(w.grid), dtype=torch.float64, device="cuda")
    wk = np.full(w.nk, 1.0 / w.nk)
    occ = np.full((w.nk, w.nbnd), 2.0)
    t = _timed(lambda: qm.qm_density(plan, -1, psi, w.nbnd, wk, occ, rho), reps)
    # algorithmic bytes per band: psi read, float64 sticks written and read back
    per_band = 16.0 * float(w.npw.mean()) + 2 * 16.0 * nst * w.grid[2]
    per_k = [w.psi(0)[:16]]
    tc = _cpu_timed(lambda: od.density_ref(w.cell, w.grid, [w.miller[0]], [1.0], [np.full(16, 2.0)], per_k))
    out["density"] = {"workload": "c3: 16 k x 160 bands -> rho on the 72^3 grid, float64",
                      "ms_per_call": 1e3 * t, "bands_per_s": bands / t,
                      "hbm": {"algorithmic_bytes_per_band": per_band,
                              "achieved_GBps": bands * per_band / t / 1e9, "peak_GBps": HBM_PEAK_GBS,
                              "frac": bands * per_band / t / 1e9 / HBM_PEAK_GBS},
                      "cpu_oracle": {"bands_per_s": 16 / tc, "cores": 1,
                                     "sample": "oracle.density.density_ref, k = 0, 16 bands"}}
    # Hartree potential: forward + inverse 3-D FFT of the grid and the Poisson multiply
    vh = torch.empty_like(rho)
    t = _timed(lambda: qm.qm_hartree(plan, rho, vh), reps)
    r_h = rho.cpu().numpy()
    tc = _cpu_timed(lambda: od.hartree_ref(w.cell, w.grid, r_h), 3)
    nr = int(np.prod(w.grid))
    # float64 complex grid read and written by each of the 3 + 3 line-FFT passes
    hb = 6 * 2 * 16.0 * nr
    out["hartree"] = {"workload": "c3: 72^3 grid, float64", "ms_per_call": 1e3 * t,
                      "hbm": {"algorithmic_bytes": hb, "achieved_GBps": hb / t / 1e9,
                              "peak_GBps": HBM_PEAK_GBS, "frac": hb / t / 1e9 / HBM_PEAK_GBS},
                      "cpu_oracle": {"ms_per_call": 1e3 * tc, "cores": 1,
                                     "sample": "oracle.density.hartree_ref on the same grid"}}
    progress("density and Hartree potential measured")
    # ETRS: nocc doubly occupied bands of every k, Taylor order 4, two steps per call
    nocc, dt, order, nsteps = 64, 0.05, 4, 2
    occ_t = np.full((w.nk, nocc), 2.0)
    flat = torch.cat([torch.from_numpy(w.psi(ik, purpose=7, nbnd=nocc).reshape(-1)) for ik in range(w.nk)]).cuda()
    vx = torch.from_numpy(w.vloc_r()).cuda()
    tstep = _timed(lambda: qm.qm_td_etrs(plan, vx, wk, occ_t, flat, nocc, dt, order, nsteps), 3) / nsteps
    happ = 3 * order * nocc * w.nk   # three exponentials of `order` H applications per band
    m0 = w.miller[0]
    b0 = w.beta(0)
    x0 = w.psi(0, purpose=7, nbnd=8)
    build = otd.hartree_model_h(w.cell, w.grid, [m0], [w.k_cryst[0]], [1.0], [np.full(8, 2.0)],
                                w.vloc_r(), [b0], w.dmat())
    tc = _cpu_timed(lambda: otd.etrs_step(build, [x0], dt, order))
    out["etrs"] = {"workload": f"c3: 16 k x {nocc} doubly occupied bands, Hartree-only model, Taylor "
                               f"order {order}, dt {dt}",
                   "ms_per_step": 1e3 * tstep, "h_band_applications_per_step": happ,
                   "h_band_applications_per_s": happ / tstep,
                   "cpu_oracle": {"ms_per_step": 1e3 * tc, "h_band_applications_per_step": 3 * order * 8,
                                  "cores": 1, "sample": "oracle.tddft.etrs_step, k = 0, 8 bands"}}
    progress("ETRS propagation measured")
    # GW matrix elements: k+q = k-point 1, k = k-point 0, 32 x 32 bands, 500 G vectors
    nb1 = nb2 = 32
    ng = 500
    ckq = torch.from_numpy(w.psi(1, purpose=5, nbnd=nb1).reshape(-1)).cuda()
    ck = torch.from_numpy(w.psi(0, purpose=6, nbnd=nb2).reshape(-1)).cuda()
    mg = w.miller[0][:ng]
    mtx = torch.empty((nb1, nb2, ng), dtype=torch.complex128, device="cuda")
    t = _timed(lambda: qm.qm_mtxel(plan, 1, ckq, nb1, 0, ck, nb2, mg, mtx), reps)
    a_kq = w.psi(1, purpose=5, nbnd=4)
    a_k = w.psi(0, purpose=6, nbnd=4)
    tc = _cpu_timed(lambda: ogw.mtxel_fft(w.grid, a_kq, w.miller[1], a_k, w.miller[0], mg))
    out["gw_mtxel"] = {"workload": f"c3: k+q = k-point 1, k = k-point 0, {nb1} x {nb2} bands, {ng} G",
                       "ms_per_call": 1e3 * t, "pairs_per_s": nb1 * nb2 / t,
                       "cpu_oracle": {"pairs_per_s": 16 / tc, "cores": 1,
                                      "sample": "oracle.gw.mtxel_fft, 4 x 4 bands, same G"}}
    progress("GW matrix elements measured")
    plan.close()
    del psi, flat, rho, vh, vx, mtx
    torch.cuda.empty_cache()
    # Hartree-only SCF to a density residual of 1e-9
    scf = {}
    for name, nocc_s, nb_s in (("c1", 1, 4), ("c2", 4, 8)):
        ws = workload.make_workload(name)
        ms, bs, vs, _ = build_inputs(ws)
        pl = qm.qm_hpsi_plan_create(ws.cell, ws.grid, ws.k_cart, ws.npw, ms, nb_s, ws.nproj, vs, bs,
                                    ws.dmat(), 0)
        start = torch.cat([torch.from_numpy(ws.psi(ik, purpose=2, nbnd=nb_s).reshape(-1))
                           for ik in range(ws.nk)]).cuda()
        r_s = torch.empty(tuple(ws.grid), dtype=torch.float64, device="cuda")
        v_s = torch.empty_like(r_s)
        kw = np.full(ws.nk, 1.0 / ws.nk)
        ps = start.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st, status = qm.qm_scf_hartree(pl, vs, kw, nocc_s, ps, nb_s, r_s, v_s, alpha=0.7, tol=1e-9)
        torch.cuda.synchronize()
        scf[name] = {"status": int(status), "s": time.perf_counter() - t0, **st}
        if name == "c1":
            beta_c1 = [bs.cpu().numpy().reshape(ws.nproj, -1)]
            tc = _cpu_timed(lambda: od.hartree_scf_ref(ws.cell, ws.grid, ws.miller, ws.k_cryst, [1.0],
                                                       ws.vloc_r(), beta_c1, ws.dmat(), nocc=1,
                                                       alpha=0.7, tol=1e-9))
            scf[name]["cpu_oracle_s"] = tc
        pl.close()
    out["scf_hartree"] = {"workload": "Hartree-only SCF, linear mixing 0.7, density residual 1e-9: "
                                      "c1 1 and c2 4 doubly occupied bands per k",
                          "runs": scf,
                          "cpu_oracle_note": "oracle.density.hartree_scf_ref (dense diagonalisation "
                                             "every iteration) on c1, one thread"}
    progress("Hartree-only SCF measured")
    return out


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--prec", default="fp64", choices=list(PREC_CODE),
                    help="precision of the reported value; the other two are measured alongside")
    ap.add_argument("--davidson", type=int, default=1,
                    help="also time the FP64 Teter Davidson to 1e-8 Ha on the Gamma + 16 k cell")
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--cpu-sample-bands", type=int, default=160)
    ap.add_argument("--other-workloads", type=int, default=1,
                    help="also measure H|psi> bands/s on the 2-, 8- and 216-atom workloads")
    ap.add_argument("--davidson-c4", type=int, default=1,
                    help="with --davidson: the arms on the 64-atom cell (0 skips them, for profiling)")
    ap.add_argument("--davidson-c5", type=int, default=1,
                    help="also time the Davidson on the 216-atom Gamma-point cell (about a minute)")
    ap.add_argument("--adjacent", type=int, default=1,
                    help="also time density, Hartree, SCF, ETRS and GW matrix elements")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first copy a MIB-sized device buffer (reference for HBM byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library runs on a single GPU "
              "(splitting the k-points over several GPUs is not implemented).", file=sys.stderr)
        sys.exit(2)

    import torch
    import workload
    import paper_2308_07277_amd as qm

    if args.copy_calibration > 0:
        src = torch.ones(args.copy_calibration * 131072, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"copy calibration: {args.copy_calibration} MiB read and written", file=sys.stderr)
        del src, dst
    w = workload.make_workload(args.workload)
    miller, beta, vloc, psi = build_inputs(w)
    plan = qm.qm_hpsi_plan_create(w.cell, w.grid, w.k_cart, w.npw, miller, w.nbnd, w.nproj,
                                  vloc, beta, w.dmat(), PREC_CODE[args.prec])
    del beta, vloc
    hpsi = torch.empty_like(psi)
    bands = w.nk * w.nbnd
    t_tune = time.perf_counter()
    qm.qm_hpsi_plan_autotune(plan, w.nbnd)
    t_tune = time.perf_counter() - t_tune

    def measure(prec):
        qm.qm_hpsi_plan_set_precision(plan, PREC_CODE[prec])
        torch.cuda.synchronize()
        for _ in range(args.warmup):
            qm.qm_apply_h(plan, -1, psi, hpsi, w.nbnd)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            qm.qm_apply_h(plan, -1, psi, hpsi, w.nbnd)
        torch.cuda.synchronize()
        ms_ = 1000.0 * (time.perf_counter() - t0) / args.steps
        st = {}
        nrep = 5
        for _ in range(nrep):
            t = qm.qm_apply_h_timed(plan, -1, psi, hpsi, w.nbnd)
            for k, v in t.items():
                st[k] = st.get(k, 0.0) + v / nrep
        return ms_, st

    others = {}
    for prec in PREC_CODE:
        if prec == args.prec:
            continue
        ms_o, st_o = measure(prec)
        others[prec] = {"bands_per_s": bands / (ms_o / 1000.0), "ms_per_step": ms_o,
                        "stages_ms": st_o}
    ms, stages = measure(args.prec)
    value = bands / (ms / 1000.0)
    model, _, nst = algorithmic_model(w, args.prec)
    dom = max(stages, key=lambda k: stages[k])
    bound, amount = model.get(dom, ("hbm", 0.0))
    sec = stages[dom] / 1000.0
    if bound == "hbm":
        achieved = amount / sec / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": recorded_traffic(w.name, args.prec, dom),
                "kernel": dom}
    elif bound == "alu":
        achieved = amount / sec / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": ALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / ALU_PEAK_TFLOPS, "traffic": recorded_traffic(w.name, args.prec, dom),
                "kernel": dom}
    else:
        dt_ = {"fp64": "f64", "fp32": "f32", "mixed": "bf16"}[args.prec]
        achieved = amount / sec / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": PEAK_TFLOPS[dt_], "unit": "TFLOP/s",
                "frac": achieved / PEAK_TFLOPS[dt_], "traffic": recorded_traffic(w.name, args.prec, dom),
                "kernel": dom}
    stage_rates = {}
    for k, (b, a) in model.items():
        if stages.get(k, 0) > 0:
            s_ = stages[k] / 1000.0
            stage_rates[k] = ({"GB/s": a / s_ / 1e9} if b == "hbm" else {"TFLOP/s": a / s_ / 1e12,
                                                                         "bound": b})
    out = {
        "metric": "Hpsi bands/s (FP64 vs mixed) + Davidson time to 1e-8 Ha residual, 64-atom",
        "value": value, "unit": "bands/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": PREC_DTYPE[args.prec], "data": "synthetic",
        "config": {"workload": f"{w.name}: {len(w.atoms)}-atom diamond-structure cell, "
                               f"{w.ecut_ry:g} Ry, {w.grid[0]}^3 grid, {w.nk} k-points, "
                               f"{w.nbnd} bands, {w.nproj} projectors, all k and bands per step",
                   "npw": [int(x) for x in w.npw], "nstick": nst, "prec": args.prec},
        "stages_ms": stages, "stage_rates": stage_rates, "roofline": roof,
        "other_precisions": others, "autotune_s": t_tune,
    }
    plan.close()
    del psi, hpsi
    torch.cuda.empty_cache()
    progress("H|psi> on the 64-atom cell measured")
    if args.other_workloads:
        out["hpsi_other_workloads"] = {}
        for n in ("c1", "c2", "c5"):
            out["hpsi_other_workloads"][n] = hpsi_rates(n)
            progress(f"H|psi> on {n} measured")
    if args.adjacent:
        out["adjacent"] = adjacent_rows()
    if args.davidson:
        weights, tinfo = train_preconditioner()
        out["mlp_training"] = tinfo
        progress("learned preconditioner trained")
        if args.davidson_c4:
            out["davidson"] = davidson_run("c4", weights=weights, oracle_k=(0, 8, 16))
            progress("Davidson on the 64-atom cell done")
        if args.davidson_c5:
            # 64 buffer bands and a 3.5x basis (1974 columns): 45 iterations instead of 70
            # with 32 buffer bands and a 3x basis, for every arm
            out["davidson_c5"] = davidson_run("c5", weights=weights, max_basis_factor=3.5,
                                              extra_bands=64,
                                              only=("fp64+teter", "fp32-ladder+teter",
                                                    "fp32-ladder+mlp"),
                                              oracle_k=(0,), oracle_bands=range(0, 500, 50))
            progress("Davidson on the 216-atom cell done")
        if args.cpu_baseline:
            out["davidson_cpu_baseline"] = davidson_cpu_baseline("c2")
            progress("Davidson CPU baseline done")
    if args.cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_sample_bands)
        progress("H|psi> CPU baseline (one thread) done")
        _, ncores = cpu_model()
        out["cpu_baseline_threaded"] = cpu_baseline(w, args.cpu_sample_bands, threads=ncores)
        progress("H|psi> CPU baseline (all cores) done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
