"""Benchmark of the batched Ewald path on one MI355X.

One step = the whole hot path over the N=1024 workload: the energy of every
walker (wrap, rho(G) in FP64, reciprocal, Jastrow and real-space sums), then a
sweep of 1024 single-electron moves per walker (move delta, accept/reject,
rho update, FP64 rho rebuild every K accepted moves in the FP32-mixed form)
through the fused multi-move call.  Inputs are seeded and synthetic and are
resident in HBM before the timed region.

Prints one JSON line.  `value` is FP32-mixed deltas/s over the whole step
(energy time included); the FP64 form is reported beside it under "fp64".
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np

METRIC = "electron-move Ewald deltas/sec at N=1024 (FP32-mixed vs FP64) + % VALU roofline"
CFG_ID = 5
PEAK_VALU_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz, FP64 and unpacked FP32
PEAK_FP32_PACKED_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0
# algorithmic work, counted as in the scope table: FMA = 2 flops
FLOP_PER_G_DELTA = 36        # two table phases (old/new), delta, t(G), weighted accumulate
FLOP_PER_PAIR_DELTA = 55     # FP64 geometry, erfc, 1/r per pair evaluation
FLOP_PER_G_PARTICLE = 10     # one phase product and one complex accumulate when rebuilding rho
FLOP_PER_PAIR_ENERGY = 55
# Jastrow p-term derivatives per G and move: rho' (2 FMA), Im/Re of conj(rho') e' (2 FMA + 2 MUL),
# a Im z (1), the three running sums (1 ADD + 2 FMA)
FLOP_PER_G_DERIV = 16
# Jastrow u term: one evaluation of the product form sum_l alpha_l r^l (r - L_u)^C costs
# N_u + C multiply-adds; a move evaluates it at the old and new distance of every partner
U_TERMS, U_C = 9, 3
FLOP_PER_U_EVAL = 2 * (U_TERMS - 1 + U_C)
# blip orbitals: 5 FMAs (value, gradient, Laplacian) per coefficient read
BLIP_WINDOW = 64


def algorithmic_flops_per_delta(n_g: int, n_part: int) -> float:
    return n_g * FLOP_PER_G_DELTA + 2 * (n_part - 1) * FLOP_PER_PAIR_DELTA


def algorithmic_flops_per_rebuild(n_g: int, n_part: int) -> float:
    return n_g * n_part * FLOP_PER_G_PARTICLE


def algorithmic_flops_per_energy(n_g: int, n_part: int) -> float:
    return algorithmic_flops_per_rebuild(n_g, n_part) + n_part * (n_part - 1) / 2 * FLOP_PER_PAIR_ENERGY


def kernel_source_hash() -> str:
    """Hash of the sources the fused kernel is compiled from."""
    csrc = os.path.join(ROOT, "paper_2507_02888_amd", "csrc")
    h = hashlib.sha256()
    for name in ("ewald_internal.h", "ewald_common.h", "ewald_run.h"):
        h.update(open(os.path.join(csrc, name), "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profiles(form: str, shape: dict):
    """Measured HBM bytes per fused launch from the committed counter summary,
    or None when it is missing, was taken on another kernel source, or on
    another launch shape (workgroup size, frame, walkers per workgroup, waves per SIMD)."""
    p = os.path.join(ROOT, "profiles", "k_run_n1024_counters.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
    except Exception:
        return None
    if d.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    for sh in d.get("shapes", []):  # one entry per profiled workgroup size
        # the queue mode (walkers_per_block > 0) is its own kernel; its traffic does not depend on the count;
        # each waves-per-SIMD bound is its own kernel too
        if (sh.get("threads") == shape.get("threads") and sh.get("general_frame", 0) == shape.get("general_frame")
                and (sh.get("walkers_per_block", 0) > 0) == (shape.get("walkers_per_block", 0) > 0)
                and sh.get("waves", 0) == shape.get("waves", 0)):
            f = sh.get("forms", {}).get(form)
            return None if f is None else f.get("hbm_bytes_per_launch")
    return None


def run_form(precision: int, batch_inputs, steps: int, warmup: int, K: int, per_step: bool = True,
             threads: int = 0, n_parity: int = 64, walkers_per_block: int = 0, waves: int = 0):
    import torch
    from paper_2507_02888_amd import ewald as ew
    cfg, b = batch_inputs["cfg"], batch_inputs["b"]
    dev = "cuda"
    sysm = cfg.systems[0]
    s = ew.System(sysm, precision=precision, refresh_every=K if precision == ew.EWALD_FP32_MIXED else 0,
                  jastrow_a=b.jastrow_a)
    batch = ew.Batch([s], b.walker_sys, device=dev)
    t = batch_inputs["tensors"]
    # launch shape: the autotuner's choice (probe sweeps on a copy of the
    # state, outside the timed region), or a fixed workgroup size
    batch.energy(t["pos"], torch.zeros(b.walkers, dtype=torch.float64, device=dev))
    if threads:
        batch.set_tuning(threads=threads, waves=waves, walkers_per_block=walkers_per_block)
    else:
        batch.autotune(n_moves=max(64, 2 * K) if precision == ew.EWALD_FP32_MIXED and K > 0 else 64)
    tuning = batch.tuning()
    W, S = b.walkers, b.steps
    energy = torch.zeros(W, dtype=torch.float64, device=dev)
    jas = torch.zeros(W, dtype=torch.float64, device=dev)
    delta = torch.zeros((S, W), dtype=torch.float64, device=dev)
    djas = torch.zeros((S, W), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        batch.energy(t["pos"], energy, jas)
        if ev is not None:
            ev[1].record(stream)
        batch.run_moves(t["k"], t["new_pos"], t["accept"], delta, djas)
        if ev is not None:
            ev[2].record(stream)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        step(evs[i])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    e_ms = [a.elapsed_time(b_) for a, b_, _ in evs]
    r_ms = [b_.elapsed_time(c) for _, b_, c in evs]
    hdr = [batch.walker_header(w) for w in (0, W // 2, W - 1)]
    n_refresh_total = None
    # every walker follows the same accept pattern statistics; count exactly
    acc_per_walker = b.accept.sum(axis=0)
    if precision == ew.EWALD_FP32_MIXED and K > 0:
        n_refresh_total = int(np.sum(acc_per_walker // K))
    else:
        n_refresh_total = 0
    assert all(h["n_refresh"] == (int(acc_per_walker[w]) // K if precision and K else 0)
               for h, w in zip(hdr, (0, W // 2, W - 1)))
    d = delta.cpu().numpy()
    assert np.all(np.isfinite(d))
    ns = min(W, n_parity)
    out = dict(elapsed=elapsed, ms_per_step=1e3 * elapsed / steps, energy_ms=float(np.mean(e_ms)),
               run_ms=float(np.mean(r_ms)), n_refresh=n_refresh_total, sample_delta=d[:4, 0].tolist(), tuning=tuning,
               drift_max=max(h["drift_max"] for h in hdr),
               # the last timed step's outputs of walkers 0..ns-1, for the parity check
               parity_sample=dict(energy=energy[:ns].cpu().numpy(), jastrow=jas[:ns].cpu().numpy(),
                                  delta=d[:, :ns].copy(), djas=djas[:, :ns].cpu().numpy()))
    if not per_step:
        batch.close()
        s.close()
        return out
    # per-step path, a short sweep of n_ps moves for its rate: move_delta +
    # accept per move, then the step call (each move's accept folded into
    # the next move's delta; the first delta and the last accept untimed)
    n_ps = min(16, S - 1)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    batch.energy(t["pos"], energy, jas)
    torch.cuda.synchronize()
    e0.record(stream)
    for m in range(n_ps):
        batch.move_delta(t["k"][m], t["new_pos"][m], delta[m], djas[m])
        batch.accept(t["accept"][m])
    e1.record(stream)
    torch.cuda.synchronize()
    out["per_step_ms_per_move"] = e0.elapsed_time(e1) / n_ps
    batch.energy(t["pos"], energy, jas)
    batch.step(None, t["k"][0], t["new_pos"][0], delta[0], djas[0])
    torch.cuda.synchronize()
    e0.record(stream)
    for m in range(1, n_ps + 1):
        batch.step(t["accept"][m - 1], t["k"][m], t["new_pos"][m], delta[m], djas[m])
    e1.record(stream)
    batch.accept(t["accept"][n_ps])
    torch.cuda.synchronize()
    out["step_ms_per_move"] = e0.elapsed_time(e1) / n_ps
    out["per_step_accept_rate"] = float(b.accept[:n_ps].mean())
    batch.close()
    s.close()
    return out


def per_step_rows(r, W: int, n_g: int, n: int, dim: int) -> dict:
    """Rates and HBM rooflines of the per-step path.  Algorithmic bytes per
    walker and move: rho read once (16 B per G of the half set) and the
    positions (8 dim N B); an accepted move (rate p) writes rho back, and the
    separate accept call reads it a second time."""
    p = r["per_step_accept_rate"]
    base = 16 * n_g + 8 * dim * n
    rows = {}
    for name, ms, nbytes, call in (
            ("two_calls", r["per_step_ms_per_move"], base + p * 2 * 16 * n_g,
             "ewald_move_delta_batch + ewald_accept_batch"),
            ("step", r["step_ms_per_move"], base + p * 16 * n_g,
             "ewald_step_batch (accept folded into the next delta)")):
        gbs = W * nbytes / (ms * 1e-3) / 1e9
        rows[name] = dict(deltas_per_s=round(W / (ms * 1e-3), 1), ms_per_move=round(ms, 4), call=call,
                          roofline=dict(bound="hbm", achieved=round(gbs, 1), peak=PEAK_HBM_GBS, unit="GB/s",
                                        frac=round(gbs / PEAK_HBM_GBS, 4), bytes_per_move=round(nbytes, 1)))
    rows["accept_rate"] = round(p, 4)
    return rows


def other_workload(cfg_id: int, precision: int, steps: int = 2, threads: int = 0, waves: int = 0):
    """A whole-workload sweep of one of the smaller configurations (energy plus
    the fused sweep, autotuned launch shape): deltas/s and the fused kernel's
    VALU fraction by the same algorithmic count."""
    import torch
    from paper_2507_02888_amd import ewald as ew
    from paper_2507_02888_amd import workloads as wl
    cfg = wl.config(cfg_id)
    b = wl.make_batch(cfg)
    mixed = precision == ew.EWALD_FP32_MIXED
    K = cfg.refresh_every if mixed else 0
    systems = [ew.System(sm, precision=precision, refresh_every=K, jastrow_a=b.jastrow_a) for sm in cfg.systems]
    batch = ew.Batch(systems, b.walker_sys, device="cuda")
    dev = "cuda"
    pos = torch.tensor(b.pos, device=dev)
    k = torch.tensor(b.k, device=dev)
    newp = torch.tensor(b.new_pos, device=dev)
    acc = torch.tensor(b.accept, device=dev)
    W, S = b.walkers, b.steps
    energy = torch.zeros(W, dtype=torch.float64, device=dev)
    delta = torch.zeros((S, W), dtype=torch.float64, device=dev)
    batch.energy(pos, energy)
    if threads:
        batch.set_tuning(threads=threads, waves=waves)
    else:
        batch.autotune(n_moves=max(64, 2 * K) if K else 64)
    stream = torch.cuda.current_stream()
    run_ms, step_ms = [], []
    for it in range(steps + 1):
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record(stream)
        batch.energy(pos, energy)
        e1.record(stream)
        batch.run_moves(k, newp, acc, delta)
        e2.record(stream)
        torch.cuda.synchronize()
        if it:  # the first pass warms up
            run_ms.append(e1.elapsed_time(e2))
            step_ms.append(e0.elapsed_time(e2))
    assert np.all(np.isfinite(delta.cpu().numpy()))
    flops = 0.0
    for w in range(W):
        si = int(b.walker_sys[w])
        sm, ng = cfg.systems[si], systems[si].info["n_g"]
        n_tot = sm.n_mobile + sm.n_fixed
        flops += S * (ng * FLOP_PER_G_DELTA + 2 * (n_tot - 1) * FLOP_PER_PAIR_DELTA)
        if K:
            flops += (int(b.accept[:, w].sum()) // K) * sm.n_mobile * ng * FLOP_PER_G_PARTICLE
    rm, sm_ = float(np.mean(run_ms)), float(np.mean(step_ms))
    out = dict(config=cfg_id, form="mixed" if mixed else "fp64", walkers=W, moves=S,
               particles=sorted({int(x.n_mobile) for x in cfg.systems}), refresh_every=K,
               deltas_per_s=round(W * S / (sm_ * 1e-3), 1), run_deltas_per_s=round(W * S / (rm * 1e-3), 1),
               launch_ms=round(rm, 4), frac=round(flops / (rm * 1e-3) / 1e12 / PEAK_VALU_TFLOPS, 4),
               launch_shape=batch.tuning())
    batch.close()
    for x in systems:
        x.close()
    return out


def timed_sweep(batch, t, delta, djas, jgrad=None, jlap=None, reps: int = 2):
    """Mean time (ms) of the fused sweep over the workload's proposals, each
    repetition from the same initial state (energy call first, untimed)."""
    import torch
    stream = torch.cuda.current_stream()
    W = delta.shape[1]
    energy = torch.zeros(W, dtype=torch.float64, device=delta.device)
    jas = None if djas is None else torch.zeros(W, dtype=torch.float64, device=delta.device)
    times = []
    for it in range(reps + 1):
        batch.energy(t["pos"], energy, jas)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        if jgrad is None:
            batch.run_moves(t["k"], t["new_pos"], t["accept"], delta, djas)  # djas may be None
        else:
            batch.run_moves_grad(t["k"], t["new_pos"], t["accept"], delta, djas, jgrad, jlap)
        e1.record(stream)
        torch.cuda.synchronize()
        if it:  # the first pass warms up
            times.append(e0.elapsed_time(e1))
    return float(np.mean(times))


def next_rows(cfg, b, t, K: int, forms=("mixed", "fp64")):
    """The rows built beyond the Ewald path, on the N=1024 workload: the
    fused sweep with the Jastrow gradient and Laplacian of every proposed
    move, and the sweep with the Jastrow two-body u term; deltas/s and the
    fused kernel's VALU fraction by the algorithmic counts above."""
    import torch
    from paper_2507_02888_amd import ewald as ew
    from paper_2507_02888_amd import workloads as wl
    sysm = cfg.systems[0]
    W, S = b.walkers, b.steps
    dev = "cuda"
    out = {}
    for form in forms:
        prec = ew.EWALD_FP32_MIXED if form == "mixed" else ew.EWALD_FP64
        kk = K if prec == ew.EWALD_FP32_MIXED else 0
        n_ref = int(np.sum(b.accept.sum(axis=0) // kk)) if kk else 0
        for row in ("jastrow_derivs", "u_term"):
            sm = wl.with_u_term(sysm, 5) if row == "u_term" else sysm
            s = ew.System(sm, precision=prec, refresh_every=kk, jastrow_a=b.jastrow_a)
            batch = ew.Batch([s], b.walker_sys, device=dev)
            batch.energy(t["pos"], torch.zeros(W, dtype=torch.float64, device=dev))
            batch.autotune(n_moves=max(64, 2 * kk) if kk else 64)
            delta = torch.zeros((S, W), dtype=torch.float64, device=dev)
            djas = torch.zeros_like(delta)
            n_g, n = s.info["n_g"], sm.n_mobile
            flops = W * S * algorithmic_flops_per_delta(n_g, n) + n_ref * algorithmic_flops_per_rebuild(n_g, n)
            if row == "jastrow_derivs":
                jg = torch.zeros((S, W, 3), dtype=torch.float64, device=dev)
                jl = torch.zeros((S, W), dtype=torch.float64, device=dev)
                ms = timed_sweep(batch, t, delta, djas, jg, jl)
                flops += W * S * n_g * FLOP_PER_G_DERIV
                del jg, jl
            else:
                ms = timed_sweep(batch, t, delta, djas)
                flops += W * S * 2 * (n - 1) * FLOP_PER_U_EVAL
            shape = batch.tuning()
            if row == "jastrow_derivs" and shape.get("threads") == 512 and shape.get("waves") == 4:
                # the tuning reports the sweep without derivatives; the
                # derivative kernels run 512-thread shapes at two waves per SIMD
                shape = dict(shape, waves=2)
            out.setdefault(row, {})[form] = dict(
                run_deltas_per_s=round(W * S / (ms * 1e-3), 1), launch_ms=round(ms, 4),
                achieved_tflops=round(flops / (ms * 1e-3) / 1e12, 3),
                frac=round(flops / (ms * 1e-3) / 1e12 / PEAK_VALU_TFLOPS, 4), launch_shape=shape)
            batch.close()
            s.close()
    out["jastrow_derivs"]["call"] = "ewald_run_moves_grad_batch (gradient and Laplacian of J per proposed move)"
    out["u_term"]["call"] = "ewald_run_moves_batch with the two-body u term (N_u = 8, C = 3, L_u = r_inscribed)"
    return out


def layers_row(forms=("mixed", "fp64"), steps: int = 2):
    """The electron-hole bilayer (two planes, Eq. (5) with z != 0; 2048
    walkers x 512 moves): ewald_run_moves_batch (the fused kernel with a
    second plane in registers, autotuned), deltas/s and its VALU fraction by
    the algorithmic count of the move (36 flops per G plus 5 for the
    cross-plane term, a dot product and a weighted add; 55 per pair evaluation) and of the mixed form's
    rebuilds; and the per-step path (move_delta + accept per call, and the
    step call that folds each accept into the next delta) for comparison,
    with its HBM fraction by the bytes it streams per move (both planes' rho
    over the half set and the positions read by the delta; the moved plane's
    rho written back by an accepted move, and read a second time by the
    separate accept call)."""
    import torch
    from paper_2507_02888_amd import ewald as ew
    from paper_2507_02888_amd import workloads as wl
    cfg = wl.bilayer_config()
    b = wl.make_batch(cfg)
    sm = cfg.systems[0]
    dev = "cuda"
    t = dict(pos=torch.tensor(b.pos, device=dev), k=torch.tensor(b.k, device=dev),
             new_pos=torch.tensor(b.new_pos, device=dev), accept=torch.tensor(b.accept, device=dev))
    W, S = b.walkers, b.steps
    out = {}
    for form in forms:
        prec = ew.EWALD_FP32_MIXED if form == "mixed" else ew.EWALD_FP64
        K = cfg.refresh_every if form == "mixed" else 0
        h = ew.System(sm, precision=prec, refresh_every=K)
        batch = ew.Batch([h], b.walker_sys, device=dev)
        e = torch.zeros(W, dtype=torch.float64, device=dev)
        batch.energy(t["pos"], e)
        batch.autotune(n_moves=max(64, 2 * K) if K else 64)
        delta = torch.zeros((S, W), dtype=torch.float64, device=dev)
        ms = timed_sweep(batch, t, delta, None, reps=steps)
        n_g, n = h.info["n_g"], sm.n_mobile
        n_ref = int(np.sum(b.accept.sum(axis=0) // K)) if K else 0
        flops = W * S * (n_g * (FLOP_PER_G_DELTA + 5) + 2 * (n - 1) * FLOP_PER_PAIR_DELTA) + \
            n_ref * algorithmic_flops_per_rebuild(n_g, n)
        # per-step path over a few moves: move_delta + accept, then the step call
        stream = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        n_ps = 16
        batch.energy(t["pos"], e)
        e0.record(stream)
        for m in range(n_ps):
            batch.move_delta(t["k"][m], t["new_pos"][m], delta[m])
            batch.accept(t["accept"][m])
        e1.record(stream)
        torch.cuda.synchronize()
        ps_ms = e0.elapsed_time(e1) / n_ps
        batch.energy(t["pos"], e)
        batch.step(None, t["k"][0], t["new_pos"][0], delta[0])
        e0.record(stream)
        for m in range(1, n_ps + 1):
            batch.step(t["accept"][m - 1], t["k"][m], t["new_pos"][m], delta[m])
        e1.record(stream)
        batch.accept(t["accept"][n_ps])
        torch.cuda.synchronize()
        st_ms = e0.elapsed_time(e1) / n_ps
        n_g = h.info["n_g"]
        p_acc = float(b.accept[:n_ps].mean())
        rows = {}
        for name, ms_m, nbytes in (("two_calls", ps_ms, 2 * 16 * n_g + 8 * 2 * n + p_acc * 2 * 16 * n_g),
                                   ("step", st_ms, 2 * 16 * n_g + 8 * 2 * n + p_acc * 16 * n_g)):
            gbs = W * nbytes / (ms_m * 1e-3) / 1e9
            rows[name] = dict(deltas_per_s=round(W / (ms_m * 1e-3), 1), ms_per_move=round(ms_m, 4),
                              roofline=dict(bound="hbm", achieved=round(gbs, 1), peak=PEAK_HBM_GBS, unit="GB/s",
                                            frac=round(gbs / PEAK_HBM_GBS, 4), bytes_per_move=round(nbytes, 1)))
        out[form] = dict(run_deltas_per_s=round(W * S / (ms * 1e-3), 1), launch_ms=round(ms, 4),
                         frac=round(flops / (ms * 1e-3) / 1e12 / PEAK_VALU_TFLOPS, 4), launch_shape=batch.tuning(),
                         per_step=rows)
        batch.close()
        h.close()
    out["call"] = ("ewald_run_moves_batch on the electron-hole bilayer (150 + 150 particles, d = 5 bohr), fused "
                   "kernel with both planes' rho in registers; per-step path beside it")
    return out


def blip_row(reps: int = 5):
    """Batched blip orbitals: 512 orbitals on a 40^3 grid over the N=1024
    cell at 65536 proposal points per call, values, gradients and
    Laplacians; points/s and the kernel's fraction of HBM bandwidth by the
    algorithmic bytes (64 coefficient rows read, 5 outputs written per
    orbital and point)."""
    import torch
    from paper_2507_02888_amd import ewald as ew
    from paper_2507_02888_amd import workloads as wl
    dev = "cuda"
    lat = wl.config(5).systems[0].lattice
    M = wl.BLIP_ORBITALS
    coef = torch.tensor(wl.blip_coefficients(), device=dev)
    pts = torch.tensor(wl.blip_points(8192, 8), device=dev)
    P = int(pts.shape[0])
    val = torch.zeros((P, M), dtype=torch.float64, device=dev)
    grad = torch.zeros((P, 3, M), dtype=torch.float64, device=dev)
    lap = torch.zeros_like(val)
    b = ew.Blips(lat, wl.BLIP_GRID, M)
    stream = torch.cuda.current_stream()
    b.eval(coef, pts, val, grad, lap)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        b.eval(coef, pts, val, grad, lap)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    bytes_per_point = BLIP_WINDOW * M * 8 + 5 * M * 8 + 24
    gbs = P * bytes_per_point / (ms * 1e-3) / 1e9
    coef_mb = coef.numel() * 8 / 1e6
    b.close()
    return dict(points_per_s=round(P / (ms * 1e-3), 1), launch_ms=round(ms, 4), points=P, orbitals=M,
                grid=list(wl.BLIP_GRID), coefficient_mb=round(coef_mb, 1),
                roofline=dict(bound="hbm", achieved=round(gbs, 1), peak=PEAK_HBM_GBS, unit="GB/s",
                              frac=round(gbs / PEAK_HBM_GBS, 4), bytes_per_point=bytes_per_point),
                call="ewald_blip_eval_batch (values, gradients, Laplacians; FP64)")


def host_threads() -> int:
    """Threads for the oracle: the OpenMP setting where the host sets one (the
    GPU host's share of its cores), else every core this process may use."""
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        return int(env)
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg, n_walkers: int, n_moves: int, threads: int):
    """The FP64 oracle on the first n_walkers walkers of the workload, OpenMP
    over walkers.  It runs twice: once with no moves (set-up, initial energy
    and rho) and once with the n_moves-move sweep; the rate is the deltas of
    the sweep over the difference of the two times.  Returns the rate and the
    oracle's outputs (the same trajectory the GPU computes)."""
    import oracle
    from paper_2507_02888_amd import workloads as wl
    b = wl.make_batch(cfg, walkers=n_walkers, moves=n_moves)
    sysm = cfg.systems[0]
    pos = b.pos.reshape(n_walkers, sysm.n_mobile, sysm.dim)
    t0 = time.perf_counter()
    oracle.run_batch(sysm, pos, b.k[:0], b.new_pos[:0], b.accept[:0], jastrow_a=b.jastrow_a, n_threads=threads)
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    r = oracle.run_batch(sysm, pos, b.k, b.new_pos, b.accept, jastrow_a=b.jastrow_a, n_threads=threads)
    t_full = time.perf_counter() - t0
    t_moves = max(t_full - t_setup, 1e-9)
    return dict(value=n_walkers * b.steps / t_moves, unit="deltas/s", cores=int(r["threads"]), kind="oracle",
                sample=f"{n_walkers} walkers x {b.steps} moves of the same workload (its first walkers, the "
                       f"trajectory the GPU computes), FP64 oracle, OpenMP over walkers on {int(r['threads'])} "
                       f"threads of a {cpu_model()}; sweep {t_moves:.1f} s wall (set-up and initial energies "
                       f"{t_setup:.1f} s, timed apart and excluded)",
                seconds=t_full + t_setup, cpu_model=cpu_model(), ref=r, n_walkers=n_walkers)


U32 = 2.0 ** -24  # FP32 unit roundoff


def mixed_djastrow_bound(system, jastrow_a, n_g_half: int) -> float:
    """Bound on the FP32-mixed form's error in a Jastrow delta dJ, from its
    arithmetic: t(G) = |rho + q d|^2 - |rho|^2 is formed in FP32 from FP32
    phases (each within ~4 units of FP32 rounding, u), so |dt| <~ 16 u |q| |rho(G)|;
    independent over the half set, the weighted sum sum_H a_s dt has a spread
    of 16 u |q| (sum_H a_s^2 |rho|^2)^(1/2) <= 16 u |q| max|a| (N_H sum_i q_i^2)^(1/2)
    for uncorrelated positions; four spreads bound the largest of many moves.
    Unlike the energy weights, the a_s do not decay with |G|, so this exceeds
    the 1e-5 of the energy deltas when N_H sum q^2 is large (N = 1024: ~7e-5).
    At least 1e-5."""
    q = np.concatenate([system.mobile_q, system.fixed_q])
    a_max = 0.0 if jastrow_a is None else float(np.max(np.abs(jastrow_a)))
    return max(1e-5, 64.0 * U32 * float(np.max(np.abs(system.mobile_q))) * a_max *
               float(np.sqrt(n_g_half * np.sum(q * q))))


def parity(form: str, got: dict, ref: dict, system, djas_bound: float = 1e-5) -> dict:
    """Largest errors of the GPU outputs against the oracle on the same walkers
    and trajectory, and whether they are within the form's bounds: FP64 1e-10
    relative (to max(|E|, (alpha/sqrt(pi)) sum q^2)) on energies and deltas;
    FP32-mixed 1e-6 relative on energies and J, 1e-5 Ha on each energy delta,
    and `djas_bound` (mixed_djastrow_bound) on each Jastrow delta."""
    q = np.concatenate([system.mobile_q, system.fixed_q])
    e_scale = system.alpha / np.sqrt(np.pi) * float(np.sum(q * q))
    n = got["energy"].shape[0]
    e_ref = ref["e0"][:n, 4]
    scale = np.maximum(np.abs(e_ref), e_scale)
    rel_e = float(np.max(np.abs(got["energy"] - e_ref) / scale))
    d_err = np.abs(got["delta"] - ref["delta"][:, :n])
    abs_d = float(np.max(d_err))
    rel_d = float(np.max(d_err / scale[None, :]))
    jscale = np.maximum(1.0, np.abs(ref["j0"][:n]))
    rel_j = float(np.max(np.abs(got["jastrow"] - ref["j0"][:n]) / jscale))
    abs_dj = float(np.max(np.abs(got["djas"] - ref["djas"][:, :n])))
    if form == "fp64":
        ok = rel_e <= 1e-10 and rel_d <= 1e-10 and rel_j <= 1e-10 and abs_dj <= 1e-10 * float(np.min(jscale))
        bounds = "energy, J: 1e-10 relative; delta, dJ: 1e-10 relative"
    else:
        ok = rel_e <= 1e-6 and abs_d <= 1e-5 and rel_j <= 1e-6 and abs_dj <= djas_bound
        bounds = f"energy, J: 1e-6 relative; delta: 1e-5 Ha; dJ: {djas_bound:.3g} (FP32 rounding of the Jastrow sum)"
    return dict(walkers=int(n), moves=int(got["delta"].shape[0]), max_rel_energy_err=rel_e,
                max_abs_delta_err=abs_d, max_rel_delta_err=rel_d, max_rel_jastrow_err=rel_j,
                max_abs_djastrow_err=abs_dj, bounds=bounds, ok=bool(ok))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--walkers", type=int, default=None, help="subset of the 8192 walkers (testing only)")
    ap.add_argument("--moves", type=int, default=None, help="subset of the 1024 moves (testing only)")
    ap.add_argument("--refresh-every", type=int, default=None)
    ap.add_argument("--cpu-walkers", type=int, default=64,
                    help="walkers of the oracle's CPU baseline, which also serve the in-run parity check")
    ap.add_argument("--cpu-threads", type=int, default=0, help="oracle threads (0: the host's share of cores)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--forms", default="mixed,fp64")
    ap.add_argument("--threads", type=int, default=0,
                    help="fixed fused-kernel workgroup size instead of the autotuner's choice")
    ap.add_argument("--walkers-per-block", type=int, default=0,
                    help="with --threads: the fused kernel's queue mode (walkers per workgroup; 0 = one each)")
    ap.add_argument("--waves", type=int, default=0,
                    help="with --threads: waves per SIMD the fused kernel is compiled for (0 = default)")
    ap.add_argument("--k-sweep", default="128,256,512,0",
                    help="further refresh intervals K timed for the mixed form (0 = no rebuild); empty to skip")
    ap.add_argument("--other", default="2,3,4",
                    help="smaller configurations also timed (both forms), reported under other_workloads")
    ap.add_argument("--next", default="derivs,u,blips,layers",
                    help="rows beyond the Ewald path also timed (jastrow derivatives, u term, blips); empty to skip")
    ap.add_argument("--skip-main", action="store_true",
                    help="time only the smaller configurations (--other) and the blip and bilayer rows named in "
                         "--next; prints their results, not the bench line")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy three times (reference for HBM counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        b_ = torch.empty_like(a)
        for _ in range(3):
            b_.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 8, "copy_bytes_written": a.numel() * 8, "copies": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported (walkers shard "
              "trivially across GPUs, but this build measures the one-GPU path)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2507_02888_amd import ewald as ew
    from paper_2507_02888_amd import workloads as wl
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    ew.load()
    if args.skip_main:
        for cid in [int(x) for x in args.other.split(",") if x]:
            for form in args.forms.split(","):
                prec = ew.EWALD_FP32_MIXED if form == "mixed" else ew.EWALD_FP64
                print(json.dumps(other_workload(cid, prec, threads=args.threads, waves=args.waves)), flush=True)
        want = set(x for x in args.next.split(",") if x)
        if "blips" in want:
            print(json.dumps({"blips": blip_row()}), flush=True)
        if "layers" in want:
            print(json.dumps({"layers": layers_row(forms=tuple(args.forms.split(",")))}), flush=True)
        return

    cfg = wl.config(CFG_ID)
    K = cfg.refresh_every if args.refresh_every is None else args.refresh_every
    b = wl.make_batch(cfg, walkers=args.walkers, moves=args.moves)
    dev = "cuda"
    tensors = dict(pos=torch.tensor(b.pos, device=dev), k=torch.tensor(b.k, device=dev),
                   new_pos=torch.tensor(b.new_pos, device=dev),
                   accept=torch.tensor(b.accept, device=dev))
    torch.cuda.synchronize()
    inputs = dict(cfg=cfg, b=b, tensors=tensors)
    sysm = cfg.systems[0]
    info = ew.System(sysm).info
    n_g, n_part = info["n_g"], sysm.n_mobile
    W, S = b.walkers, b.steps
    deltas_per_step = W * S

    results = {}
    for form in args.forms.split(","):
        prec = ew.EWALD_FP32_MIXED if form == "mixed" else ew.EWALD_FP64
        r = run_form(prec, inputs, args.steps, args.warmup, K, threads=args.threads, n_parity=args.cpu_walkers,
                     walkers_per_block=args.walkers_per_block, waves=args.waves)
        flops_run = deltas_per_step * algorithmic_flops_per_delta(n_g, n_part) + \
            r["n_refresh"] * algorithmic_flops_per_rebuild(n_g, n_part)
        achieved = flops_run / (r["run_ms"] * 1e-3) / 1e12
        traffic = traffic_from_profiles(form, r["tuning"])
        r["value"] = deltas_per_step / (r["ms_per_step"] * 1e-3)
        r["roofline"] = dict(bound="alu", achieved=round(achieved, 3), peak=PEAK_VALU_TFLOPS, unit="TFLOP/s",
                             frac=round(achieved / PEAK_VALU_TFLOPS, 4), traffic=traffic,
                             kernel=f"k_run ({form}), fused {S}-move sweep of {W} walkers",
                             launch_shape=r["tuning"],
                             flop_per_launch=flops_run, launch_ms=round(r["run_ms"], 4),
                             frac_of_packed_fp32_peak=round(achieved / PEAK_FP32_PACKED_TFLOPS, 4)
                             if form == "mixed" else None)
        e_flops = W * algorithmic_flops_per_energy(n_g, n_part)
        r["energies_per_s"] = W / (r["energy_ms"] * 1e-3)
        r["energy_kernel"] = dict(ms=round(r["energy_ms"], 4), achieved_tflops=round(e_flops / (r["energy_ms"] * 1e-3) / 1e12, 3))
        r["per_step_deltas_per_s"] = W / (r["per_step_ms_per_move"] * 1e-3)
        r["per_step"] = per_step_rows(r, W, n_g, n_part, sysm.dim)
        results[form] = r

    sweep = []
    if "mixed" in results and args.k_sweep:
        for k_alt in [int(x) for x in args.k_sweep.split(",")]:
            r = run_form(ew.EWALD_FP32_MIXED, inputs, max(1, min(args.steps, 2)), 1, k_alt, per_step=False,
                         threads=args.threads)
            flops_run = deltas_per_step * algorithmic_flops_per_delta(n_g, n_part) + \
                r["n_refresh"] * algorithmic_flops_per_rebuild(n_g, n_part)
            sweep.append(dict(refresh_every=k_alt, run_deltas_per_s=round(deltas_per_step / (r["run_ms"] * 1e-3), 1),
                              launch_ms=round(r["run_ms"], 4), rebuilds=r["n_refresh"],
                              frac=round(flops_run / (r["run_ms"] * 1e-3) / 1e12 / PEAK_VALU_TFLOPS, 4),
                              drift_max=r["drift_max"] if k_alt > 0 else None))

    nxt = {}
    want = set(x for x in args.next.split(",") if x)
    if want & {"derivs", "u"}:
        nxt.update(next_rows(cfg, b, tensors, K, forms=tuple(f for f in args.forms.split(","))))
    if "blips" in want:
        nxt["blips"] = blip_row()
    if "layers" in want:
        nxt["layers"] = layers_row(forms=tuple(f for f in args.forms.split(",")))

    others = []
    if args.other:
        for cid in [int(x) for x in args.other.split(",")]:
            for prec in (ew.EWALD_FP32_MIXED, ew.EWALD_FP64):
                others.append(other_workload(cid, prec))

    cpu = None
    parity_ok = True
    if not args.no_cpu:
        cpu = cpu_baseline(cfg, min(args.cpu_walkers, W), S, args.cpu_threads or host_threads())
        for form, r in results.items():
            r["parity"] = parity(form, r["parity_sample"], cpu["ref"], sysm,
                                 mixed_djastrow_bound(sysm, b.jastrow_a, n_g))
            parity_ok &= r["parity"]["ok"]

    head = results.get("mixed") or results[next(iter(results))]
    line = {
        "metric": METRIC,
        "value": round(head["value"], 1),
        "unit": "deltas/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-mixed" if "mixed" in results else "f64",
        "data": "synthetic",
        "config": {"workload": f"3D electron gas, bcc-shaped cell, N={n_part} at rs=1, {W} walkers x {S} "
                               f"moves per step, |G|<=12(2pi/L) ({n_g} G in the half set), Jastrow "
                               f"plane-wave term, FP64 rho rebuild every {K} accepts (mixed form)",
                   "walkers": W, "moves_per_walker": S, "particles": n_part, "n_g_half": n_g,
                   "refresh_every": K, "call": "ewald_energy_batch + ewald_run_moves_batch"},
        "roofline": head["roofline"],
        "cpu_baseline": None if cpu is None else {k: cpu[k] for k in ("value", "unit", "cores", "kind", "sample")},
        "parity": None if cpu is None else head.get("parity"),
        "energies_per_s": round(head["energies_per_s"], 1),
        "per_step_path_deltas_per_s": round(head["per_step"]["step"]["deltas_per_s"], 1),
        "per_step": head["per_step"],
    }
    if sweep:
        k_main = results["mixed"]
        line["mixed_refresh_sweep"] = [dict(refresh_every=K, run_deltas_per_s=round(deltas_per_step / (k_main["run_ms"] * 1e-3), 1),
                                            launch_ms=round(k_main["run_ms"], 4), rebuilds=k_main["n_refresh"],
                                            frac=k_main["roofline"]["frac"], drift_max=k_main["drift_max"])] + sweep
    if others:
        line["other_workloads"] = others
    if nxt:
        line["next_rows"] = nxt
    if "fp64" in results and "mixed" in results:
        f = results["fp64"]
        line["fp64"] = {"value": round(f["value"], 1), "unit": "deltas/s", "ms_per_step": round(f["ms_per_step"], 3),
                        "roofline": f["roofline"], "energies_per_s": round(f["energies_per_s"], 1),
                        "per_step_path_deltas_per_s": round(f["per_step"]["step"]["deltas_per_s"], 1),
                        "per_step": f["per_step"], "parity": f.get("parity")}
    if os.environ.get("EWALD_TIMING", "0") not in ("", "0"):
        line["call_timers"] = ew.ewald_timing_report()  # per ABI call, over the whole run (warm-up included)
    print(json.dumps(line), flush=True)
    if not parity_ok:
        print("bench.py: GPU results differ from the oracle beyond the stated bounds", file=sys.stderr)
        sys.exit(3)


if __name__ == "__main__":
    main()
