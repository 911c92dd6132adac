#!/usr/bin/env python3
"""Benchmark of the spectral flame step on one MI355X.

One bench step is one integrating-factor Euler step of Eq. (1) for the
2048 x 4096 flame (row kernel + column kernel), with the FP64 diagnostic
reductions every 50 steps as in that workload. Inputs are resident in HBM
before the timed region starts. Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
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

HBM_PEAK_GBS = 8000.0
# MI355X FP32 vector peak (256 CUs x 4 SIMDs x 16 lanes x 2 flops per FMA x 2
# for packed FP32 x 2.4 GHz); without packed FP32 instructions half of it
FP32_VECTOR_PEAK_TFLOPS = 157.3
CIRCLE_SOURCES = ("paper_0911_2889_amd/csrc/circle_kernels.hip", "paper_0911_2889_amd/csrc/fft_engine.hpp",
                  "paper_0911_2889_amd/csrc/flame_dev.hpp",
                  "paper_0911_2889_amd/csrc/kernel_common.hpp")
KERNEL_SOURCES = ("paper_0911_2889_amd/csrc/flame_kernels.hip", "paper_0911_2889_amd/csrc/step_bodies.hpp",
                  "paper_0911_2889_amd/csrc/fft_engine.hpp", "paper_0911_2889_amd/csrc/flame_dev.hpp",
                  "paper_0911_2889_amd/csrc/kernel_common.hpp")


def algorithmic_bytes(n1, n2, rows=None, forcing=False):
    """Bytes each kernel of one step must move (FP32 complex = 8 bytes), with
    the quadratic term formed on `rows` theta rows (n1, or 3*n1/4 on the
    product grid; default n1).

    row: read the column-transformed gradient spectrum rows x (2K2+1), write
         the row transform of |grad Phi|^2, rows x (K2+1);
    col: read that rows x (K2+1), read and write the state (2K1+1) x (K2+1),
         write the next gradient spectrum rows x (2K2+1); with a forcing,
         also read the forcing spectrum (2K1+1) x (K2+1).
    """
    rows = n1 if rows is None else rows
    k1, k2 = (n1 - 1) // 4, (n2 - 1) // 4
    row = 8 * (rows * (2 * k2 + 1) + rows * (k2 + 1))
    col = 8 * (rows * (k2 + 1) + (3 if forcing else 2) * (2 * k1 + 1) * (k2 + 1) + rows * (2 * k2 + 1))
    return {"row": row, "col": col}


def row_pass_flops(rows, cols):
    """Nominal flops of one row pass (the row kernel's launch): per grid row the
    inverse complex transform of the packed gradient (5 L log2 L on L = cols
    points), |z|^2 (3 per point) and half of the forward complex transform that
    serves two real rows (2.5 L log2 L)."""
    lg = math.log2(cols)
    return rows * (5.0 * cols * lg + 3.0 * cols + 2.5 * cols * lg)


# store kinds of flame_set_streaming_stores: names on the command line and in the record
STORE_KINDS = {"plain": 0, "streaming": 1, "nt-w": 2, "nt-q": 3}
STORE_KIND_NAMES = {0: "plain", 1: "streaming", 2: "nt-w", 3: "nt-q"}


def source_digest():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload, pts, rows, streaming=0):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources and lists the same variant of the
    kernel (points per thread, product-grid rows, and a store-kind code of
    flame_set_streaming_stores that runs it: `streaming_codes`, or one
    `streaming` code where true stands for 1); else None."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_kernel_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_digest") != source_digest():
        return None
    for v in rec.get("variants", []):
        codes = v.get("streaming_codes", [int(v.get("streaming", 0))])
        if v.get("points_per_thread") == pts and v.get("rows") == rows and streaming in codes:
            return v.get("hbm_bytes_per_launch")
    return None


def host_cores():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def circle_record(path=os.path.join(ROOT, "profiles", "circle_kernel_circles4096x2048_valu.json")):
    """VALU instructions per wave and step of the circle kernel from the
    committed counter record, if it was taken on the current circle sources."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    h = hashlib.sha256()
    for rel in CIRCLE_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return rec if rec.get("source_digest") == h.hexdigest()[:16] else None


def cpu_oracle_baseline(w, half, seconds, workers=None):
    """Time the FP64 oracle on the host on a bounded sample of the same
    workload: numpy's single-threaded transforms (workers None), or scipy.fft
    with `workers` threads (oracle.set_fft_workers)."""
    import numpy as np

    import oracle

    p = oracle.Params(w.n1, w.n2, gamma=w.gamma, theta_pi=w.theta_pi, t0=w.t0, dt=w.dt)
    cur = oracle.run(oracle.half_to_full(half.astype(np.complex128), w.n1, w.n2), p, 0)
    steps = 0
    oracle.set_fft_workers(workers)
    try:
        t0 = time.perf_counter()
        while True:
            cur = oracle.step(cur, p, steps)
            steps += 1
            el = time.perf_counter() - t0
            if el >= seconds or steps >= w.steps:
                break
    finally:
        oracle.set_fft_workers(None)
    fft = "single-threaded numpy pocketfft" if workers is None else f"scipy.fft, {workers} workers"
    return {
        "value": w.points * steps / el,
        "unit": "point-steps/s",
        "cores": 1 if workers is None else workers,
        "kind": "oracle",
        "sample": f"first {steps} steps of {w.name} from its initial condition, FP64 ({fft}), {el:.1f} s",
        "host_cpu_count": os.cpu_count(),
        "host_affinity": host_cores(),
    }, steps, oracle.full_to_half(cur, w.n1, w.n2)


def copy_bandwidth(nbytes, reps=20):
    """Read + write GB/s of a plain device copy of nbytes (torch copy kernel), HIP events."""
    import torch

    n = nbytes // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    return 2.0 * n * 4 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9


def copy_sweep(mib=(8, 16, 32, 48, 64, 128, 256, 512), reps=50, trials=5):
    """Read + write GB/s of plain device copies by size, each timed over a
    hipGraph replay of `reps` copies (best of `trials`), so that launch gaps do
    not count. Source and destination together up to the Infinity Cache's
    256 MB stay resident there; larger copies stream from HBM."""
    import torch

    out = {}
    for m in mib:
        n = m * 1024 * 1024 // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for _ in range(3):
                dst.copy_(src)
        torch.cuda.current_stream().wait_stream(side)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for _ in range(reps):
                dst.copy_(src)
        g.replay()
        torch.cuda.synchronize()
        best = 0.0
        for _ in range(trials):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            g.replay()
            e1.record()
            torch.cuda.synchronize()
            best = max(best, 2.0 * n * 4 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9)
        out[str(m)] = round(best, 1)
        del g, src, dst
    return out


def adjoint_leg(steps, every, reps=2):
    """Checkpointed gradient of the area excess on the adjoint workload: HIP-event
    time of the forward pass (projection, steps, diagnostics) and of the backward
    pass (seed, segment recomputation, adjoint steps, synthesis)."""
    import torch

    import synth
    from paper_0911_2889_amd import FlameSim, flame_area

    w = synth.WORKLOADS["adjoint1024x2048"]
    sim = FlameSim(w.n1, w.n2, gamma=w.gamma, theta_pi=w.theta_pi, t0=w.t0, dt=w.dt)
    sim.set_spectrum(synth.workload_spectrum(w))
    phi0 = sim.phi().clone()
    fwd, bwd = [], []
    for r in range(reps + 1):
        x = phi0.clone().requires_grad_(True)
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        torch.cuda.synchronize()
        e0.record()
        J = flame_area(x, sim, steps, checkpoint_every=every)
        e1.record()
        J.backward()
        e2.record()
        torch.cuda.synchronize()
        if r:  # the first repetition warms up
            fwd.append(e0.elapsed_time(e1))
            bwd.append(e1.elapsed_time(e2))
    f, b = min(fwd), min(bwd)
    return {
        "workload": w.name, "grid": [w.n1, w.n2], "steps": steps, "checkpoint_every": every,
        "forward_ms": f, "backward_ms": b, "backward_over_forward": b / f,
        "adjoint_point_steps_per_s": w.points * steps / (b * 1e-3),
        "forward_point_steps_per_s": w.points * steps / (f * 1e-3),
        "J": J.item(),
    }


def forced_leg(sim, w, half, steps, graph_steps, run_steps, unforced_ms, rows):
    """The same flame with a seeded forcing f~ bound (every mode of the box,
    amplitude 1e-5/|k|): HIP-event time of `steps` steps in the launch
    configuration of the main measurement, then per-kernel times of direct
    launches. The forcing is removed afterwards."""
    import torch

    import synth

    sim.set_forcing(synth.forcing_spectrum(w, amp=1e-5))
    sim.set_spectrum(half)
    run_steps(max(steps // 4, graph_steps), False)  # warm-up
    sim.set_spectrum(half)
    sim.step(0)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    run_steps(steps, False)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    saved = graph_steps
    sim.set_graph_steps(0)
    sim.set_spectrum(half)
    sim.step(0)
    kt = run_steps(steps, True)
    torch.cuda.synchronize()
    sim.set_graph_steps(saved)
    sim.set_forcing(None)
    nbytes = algorithmic_bytes(w.n1, w.n2, rows, forcing=True)
    col_ms = kt["col"][0] / max(1, kt["col"][1])
    return {
        "forcing": "every mode of the box, amp 1e-5/|k|, seed workload seed + 7919",
        "steps": steps, "ms_per_step": ms, "point_steps_per_s": w.points / (ms * 1e-3),
        "over_unforced": ms / unforced_ms,
        "step_bytes": nbytes["row"] + nbytes["col"],
        "step_hbm_frac": (nbytes["row"] + nbytes["col"]) / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "col_kernel_ms": col_ms, "col_kernel_GB_s": nbytes["col"] / (col_ms * 1e-3) / 1e9,
        "kernels_ms_per_step": {k: kt[k][0] / max(1, steps) for k in ("row", "col", "diag")},
    }


def heun_leg(w, half, steps, graph_steps, diag_every, euler_ms):
    """The same workload stepped with integrating-factor Heun (two row and two
    column kernels per step) on its own plan, autotuned, graph replays between
    diagnostics: HIP-event time of `steps` steps, then per-kernel times of
    direct launches."""
    import torch

    from paper_0911_2889_amd import FlameSim

    sim = FlameSim(w.n1, w.n2, gamma=w.gamma, theta_pi=w.theta_pi, t0=w.t0, dt=w.dt, integrator=1)
    sim.set_spectrum(half)
    sim.autotune(steps=20)
    pts = sim.points_per_thread(w.n1, w.n2)
    rows = 3 * w.n1 // 4 if sim.product_grid(w.n1, w.n2) else w.n1
    diag = torch.zeros(4, dtype=torch.float64, device=sim.device)

    def run(k, timed):
        if timed:
            sim.timing_begin()
        done = 0
        while done < k:
            chunk = min(diag_every - (done % diag_every), k - done)
            sim.step(chunk)
            done += chunk
            if done % diag_every == 0:
                sim.diagnostics(out=diag)
        return sim.timing_end() if timed else None

    sim.set_graph_steps(graph_steps)
    sim.set_spectrum(half)
    run(max(graph_steps, 10), False)  # warm-up (builds the graph)
    sim.set_spectrum(half)
    sim.step(0)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    run(steps, False)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    sim.set_graph_steps(0)
    sim.set_spectrum(half)
    sim.step(0)
    kt = run(steps, True)
    torch.cuda.synchronize()
    nb = algorithmic_bytes(w.n1, w.n2, rows)
    k1, k2 = (w.n1 - 1) // 4, (w.n2 - 1) // 4
    step_bytes = 2 * nb["row"] + 2 * nb["col"] + 8 * (2 * k1 + 1) * (k2 + 1)  # the corrector also reads Phi*
    return {
        "integrator": "integrating-factor Heun (2 row + 2 column kernels per step)",
        "steps": steps, "graph_steps": graph_steps, "points_per_thread": {"col": pts[0], "row": pts[1]},
        "product_rows": rows, "streaming_stores": sim.streaming_stores(w.n1, w.n2), "ms_per_step": ms,
        "point_steps_per_s": w.points / (ms * 1e-3), "over_euler": ms / euler_ms, "step_bytes": step_bytes,
        "step_hbm_frac": step_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "kernels_ms_per_launch": {k: kt[k][0] / max(1, kt[k][1]) for k in ("row", "col")},
    }


def power_law_fit(ts, v, t_from, t_star_lo=-2000.0, step=5.0):
    """Least-squares fit of log v = log A + alpha log(t - t*) over t >= t_from,
    with t* scanned on [t_star_lo, t_from)."""
    import numpy as np

    sel = (ts >= t_from) & (v > 0) & np.isfinite(v)
    if sel.sum() < 4:
        return None
    y = np.log(v[sel])
    best = None
    for tstar in np.arange(t_star_lo, t_from, step):
        a = np.vstack([np.ones(int(sel.sum())), np.log(ts[sel] - tstar)]).T
        coef = np.linalg.lstsq(a, y, rcond=None)[0]
        rms = float(np.sqrt(np.mean((a @ coef - y) ** 2)))
        if best is None or rms < best["rms_log_residual"]:
            best = {"alpha": float(coef[1]), "t_star": float(tstar), "rms_log_residual": rms,
                    "window": [float(t_from), float(ts[sel][-1])]}
    return best


def long_run_leg(n=8192, t_end=2600.0, dt=0.1, every_t=5.0, fits_from=(1500.0,)):
    """Long-horizon run in the setting of Section 2's spherical-flame runs:
    node noise eps*eta, eps = 1e-3, t0 = 200, gamma = 0.8, no forcing, on an
    n x n grid with integrating-factor Heun, diagnostics every `every_t`, and
    power-law fits <Phi_t> ~ A (t - t*)^alpha over t >= each of fits_from.
    Qualitative: the paper quotes alpha ~ 0.76 over an unstated interval and
    grid."""
    import numpy as np
    import torch

    import synth
    from paper_0911_2889_amd import FlameSim

    every = int(round(every_t / dt))
    sim = FlameSim(n, n, gamma=0.8, theta_pi=1.0, t0=200.0, dt=dt, integrator=1)
    sim.set_phi(synth.physical_noise(n, n, seed=0, kind="uniform", scale=1e-3))
    sim.autotune(steps=3)  # leaves the state and the step index as they are
    sim.set_graph_steps(every)
    nd = int(round((t_end - 200.0) / dt)) // every
    diag = torch.zeros((nd, 4), dtype=torch.float64, device=sim.device)
    torch.cuda.synchronize()
    t_wall = time.time()
    for i in range(nd):
        sim.step(every)
        sim.diagnostics(out=diag[i])
    torch.cuda.synchronize()
    wall = time.time() - t_wall
    d = diag.cpu().numpy()
    ts = 200.0 + dt * every * np.arange(1, nd + 1)
    bad = np.nonzero(d[:, 3] == 0)[0]
    good = d[:, 3] == 1
    stride = max(1, int(round(100.0 / every_t)))
    return {
        "setting": "node noise eps*eta (eps 1e-3, seed 0), t0 200, gamma 0.8, f = 0 (Section 2)",
        "grid": [n, n], "integrator": "integrating-factor Heun", "dt": dt, "t_end": t_end,
        "points_per_thread": list(sim.points_per_thread(n, n)), "product_grid": sim.product_grid(n, n),
        "store_kind": STORE_KIND_NAMES[sim.streaming_stores(n, n)],
        "steps": nd * every, "wall_s": wall, "point_steps_per_s_with_diagnostics": n * n * nd * every / wall,
        "first_nonfinite_t": float(ts[bad[0]]) if len(bad) else None,
        "series_every_100": {"t": ts[stride - 1::stride].tolist(), "velocity": d[stride - 1::stride, 1].tolist(),
                             "mean_radius": d[stride - 1::stride, 0].tolist(),
                             "area_excess": d[stride - 1::stride, 2].tolist()},
        "power_law_fits": [power_law_fit(ts[good], d[good, 1], t_from) for t_from in fits_from],
        # the same with t* fixed at 0 (t* and alpha trade off strongly over short windows)
        "power_law_fits_t_star_0": [power_law_fit(ts[good], d[good, 1], t_from, t_star_lo=0.0, step=t_from)
                                    for t_from in fits_from],
    }


# One wave-instruction per CU per clock (4 SIMDs x 16 lanes, wave64, FP32
# not packed): the vector-ALU issue peak of 256 CUs at 2.4 GHz, and its FP32
# rate (an FMA is 2 flops per lane), half of the packed FP32 peak above; the
# kernels here are built without packed FP32 instructions.
VALU_PEAK_INSTR_S = 256 * 2.4e9
FP32_UNPACKED_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12


def circle_leg(n=4096, count=2048, steps=200, valu_per_wave_step=None):
    """Batched circular flames (the one-dimensional Eq. (1)): `count` circles
    of n points stepped `steps` times in one launch, timed with in-dispatch
    order HIP events. Roofline: vector ALU (the spectra stay in registers).
    valu_per_wave_step: VALU instructions per wave per step from the counter
    record (profiles/circle_kernel_*.md), for the issue fraction."""
    import math

    import torch

    import synth
    from paper_0911_2889_amd import CircleBatch

    b = CircleBatch(n, count, t0=200.0, dt=0.25)
    spec = synth.circle_spectra(n, count, seed=7, amp=1e-3)
    b.set_spectra(spec)
    b.step(20)  # warm-up
    b.set_spectra(spec)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    b.step(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    pairs = (count + 1) // 2
    # nominal FFT flops: one inverse and one forward complex transform of n points per pair and step
    flops = pairs * steps * 2 * 5.0 * n * math.log2(n)
    out = {"circles": count, "points": n, "steps": steps, "ms": ms, "us_per_step": ms * 1e3 / steps,
           "point_steps_per_s": n * count * steps / (ms * 1e-3),
           "nominal_fft_tflops": flops / (ms * 1e-3) / 1e12,
           "fp32_vector_peak_tflops": FP32_VECTOR_PEAK_TFLOPS,
           "nominal_frac": flops / (ms * 1e-3) / 1e12 / FP32_VECTOR_PEAK_TFLOPS,
           "nominal_frac_of_unpacked_peak": flops / (ms * 1e-3) / 1e12 / FP32_UNPACKED_PEAK_TFLOPS}
    if valu_per_wave_step:
        g = n // 16
        per_wg = max(1, 256 // g)  # circle pairs per workgroup
        waves = -(-pairs // per_wg) * (per_wg * g) // 64
        rate = valu_per_wave_step * waves * steps / (ms * 1e-3)
        out["valu_per_wave_step"] = valu_per_wave_step
        out["valu_issue_frac"] = rate / VALU_PEAK_INSTR_S
    return out


def circle_long_run_leg(n=8192, count=64, t_end=4000.0, dt=0.1, every_t=5.0, fits_from=(1500.0, 2500.0)):
    """Long run of circular flames (Section 2's comparison of spherical with
    circular flames): `count` circles of n points from seeded modal noise of
    amplitude 1e-3 at t0 = 200, gamma = 0.8, integrating-factor Euler,
    averages every `every_t`; the batch-mean <Phi_t> fitted by
    A (t - t*)^alpha over t >= each of fits_from. Qualitative: the paper
    reports that circular flames settle to alpha = 1/4."""
    import numpy as np
    import torch

    import synth
    from paper_0911_2889_amd import CircleBatch

    every = int(round(every_t / dt))
    b = CircleBatch(n, count, t0=200.0, dt=dt)
    b.set_spectra(synth.circle_spectra(n, count, seed=11, amp=1e-3))
    nd = int(round((t_end - 200.0) / dt)) // every
    diag = torch.zeros((nd, count, 4), dtype=torch.float64, device=b.device)
    torch.cuda.synchronize()
    t_wall = time.time()
    for i in range(nd):
        b.step(every)
        b.diagnostics(out=diag[i])
    torch.cuda.synchronize()
    wall = time.time() - t_wall
    d = diag.cpu().numpy()
    ts = 200.0 + dt * every * np.arange(1, nd + 1)
    ok = (d[:, :, 3] == 1).all(axis=1)
    vel = d[:, :, 1].mean(axis=1)
    stride = max(1, int(round(100.0 / every_t)))
    return {
        "setting": f"{count} circles, modal noise amp 1e-3 (seed 11), t0 200, gamma 0.8, f = 0, IF-Euler",
        "points": n, "dt": dt, "t_end": t_end, "steps": nd * every, "wall_s": wall,
        "point_steps_per_s_with_diagnostics": n * count * nd * every / wall,
        "first_nonfinite_t": float(ts[~ok][0]) if (~ok).any() else None,
        "series_every_100": {"t": ts[stride - 1::stride].tolist(), "velocity": vel[stride - 1::stride].tolist()},
        "power_law_fits": [power_law_fit(ts[ok], vel[ok], t_from) for t_from in fits_from],
    }


def use_persistent_config(ens, grids):
    """Put every grid group of an ensemble on the persistent kernel's
    configuration: product grid, 12 column and 16 row points per thread, plain
    stores, whatever the autotuner chose before (the product grid first: the
    12-point column kernels need it)."""
    for n1, n2 in grids:
        ens.set_product_grid(n1, n2, True)
        ens.set_points_per_thread(n1, n2, 12, 16)
        ens.set_streaming_stores(n1, n2, False)


def ensemble_leg(steps, graph_steps):
    """The batched ensemble (256 flames of three grids) stepped in graphs of
    graph_steps steps, and with direct launches, timed with HIP events."""
    import torch

    import synth
    from paper_0911_2889_amd import FlameEnsemble

    members = synth.ensemble_members()
    descs = [dict(n1=w.n1, n2=w.n2, gamma=w.gamma, theta_pi=w.theta_pi, t0=w.t0, dt=w.dt) for w in members]
    ens = FlameEnsemble(descs)
    halves = [synth.workload_spectrum(w) for w in members]
    points = sum(w.points for w in members)
    nbytes = None  # set after autotuning, which picks each group's grid
    for f, h in enumerate(halves):
        ens.set_spectrum(h, flame=f)
    ens.set_graph_steps(graph_steps)
    # per grid group, then jointly for the groups' concurrent graph branches; with 10 timed
    # steps per trial the choices followed timing noise and the replayed step was ~3 % slower
    ens.autotune(steps=30)
    grids = ((128, 256), (256, 512), (512, 1024))
    tuned = {f"{n1}x{n2}": list(ens.points_per_thread(n1, n2)) + ["product" if ens.product_grid(n1, n2) else "n1"]
             + [STORE_KIND_NAMES[ens.streaming_stores(n1, n2)]] for n1, n2 in grids}
    nbytes = sum(sum(algorithmic_bytes(w.n1, w.n2, 3 * w.n1 // 4 if ens.product_grid(w.n1, w.n2) else w.n1).values())
                 for w in members)
    out = {"flames": len(members), "grids": "128 x 128x256, 96 x 256x512, 32 x 512x1024", "steps": steps,
           "timing": "median of 3 back-to-back timed runs of `steps` steps after 200 untimed ones",
           "warmup_steps": 200,
           "points": points, "step_bytes": nbytes, "points_per_thread": tuned}

    def timed(warm, runs=3):
        # steady state: the initial states, `warm` untimed steps (they build the
        # graph or the persistent partition; the first hundreds of steps after a
        # pause run ~6 % slower), then the median of `runs` back-to-back timed
        # runs of `steps` steps
        for f, h in enumerate(halves):
            ens.set_spectrum(h, flame=f)
        ens.step(warm)
        torch.cuda.synchronize()
        per_run = []
        for _ in range(runs):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            ens.step(steps)
            e1.record()
            torch.cuda.synchronize()
            per_run.append(e0.elapsed_time(e1))
        ms = sorted(per_run)[len(per_run) // 2]
        return {"ms_per_step": ms / steps, "point_steps_per_s": points * steps / (ms * 1e-3),
                "step_hbm_frac": nbytes / (ms / steps * 1e-3) / 1e9 / HBM_PEAK_GBS,
                "ms_per_step_runs": [t / steps for t in per_run]}

    for mode, gs in (("graph", graph_steps), ("direct", 0)):
        ens.set_graph_steps(gs)
        out[mode] = timed(200)
    # A/B of the persistent launch: every group on the persistent kernel's
    # configuration (product grid, 12 column and 16 row points per thread,
    # plain stores), against graph replays of the same kernels' bodies
    use_persistent_config(ens, grids)
    ens.set_graph_steps(graph_steps)
    out["graph_persistent_config"] = timed(200)
    ens.set_graph_steps(0)
    runs = {}
    for wgs in (0, 256):
        ens.set_persistent(True, workgroups=wgs)
        r = timed(200)
        r["workgroups"] = ens.persistent()[1]
        runs[wgs] = r
    best = min(runs.values(), key=lambda r: r["ms_per_step"])
    out["persistent"] = dict(best, grids_tried={str(r["workgroups"]): r["ms_per_step"] for r in runs.values()})
    # the same launch captured in a graph of graph_steps steps (counter reset
    # node + cooperative kernel node), replayed
    ens.set_persistent(True, workgroups=best["workgroups"])
    ens.set_graph_steps(graph_steps)
    out["persistent_graph"] = dict(timed(200), workgroups=ens.persistent()[1], graph_steps=graph_steps)
    ens.set_persistent(False)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="flame2048x4096")
    ap.add_argument("--diag-every", type=int, default=50)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--pts", type=int, nargs=2, metavar=("COL", "ROW"),
                    help="points per thread of the column and row step kernels (default: autotuned)")
    ap.add_argument("--no-graph", action="store_true", help="launch every step directly (no hipGraph replays)")
    ap.add_argument("--grid", choices=("product", "n1"),
                    help="form the quadratic term on 3*N1/4 rows or on N1 rows (default: autotuned)")
    ap.add_argument("--stores", choices=tuple(STORE_KINDS),
                    help="store kind of the step's intermediates Q and W: plain, non-temporal for both "
                         "('streaming'), for W only or for Q only (default: autotuned)")
    ap.add_argument("--ensemble-steps", type=int, default=200,
                    help="steps of the 256-flame ensemble leg (0 skips it)")
    ap.add_argument("--forcing-steps", type=int, default=200,
                    help="steps of the forced-step leg (a seeded forcing bound to the same flame); 0 skips it")
    ap.add_argument("--heun-steps", type=int, default=200,
                    help="steps of the integrating-factor Heun leg on the same workload; 0 skips it")
    ap.add_argument("--no-long-run", action="store_true",
                    help="skip the long-horizon run (8192 x 8192, Heun, t = 200 .. 2600)")
    ap.add_argument("--long-run-t-end", type=float, default=2600.0,
                    help="end time of the long-horizon run (a shorter one serves profiling of its kernels)")
    ap.add_argument("--adjoint-steps", type=int, default=100,
                    help="steps of the checkpointed adjoint leg on 1024x2048 (0 skips it)")
    ap.add_argument("--circle-steps", type=int, default=200,
                    help="steps of the batched circular-flame leg (2048 circles of 4096 points; 0 skips it)")
    ap.add_argument("--no-circle-long-run", action="store_true",
                    help="skip the long run of 64 circular flames of 8192 points to t = 4000")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES bytes 5 times (calibrates HBM counters)")
    ap.add_argument("--copy-sweep", action="store_true",
                    help="only measure plain device copies of 8 MiB .. 512 MiB (graph replays of 50 copies) "
                         "and print their read + write GB/s")
    args = ap.parse_args()

    if args.copy_sweep:
        print(json.dumps({"copy_sweep_GB_s": copy_sweep()}))
        return

    if args.copy_probe:
        import torch

        n = args.copy_probe // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n * 4}))
        return

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(the multi-GPU slab decomposition is described, not implemented)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_0911_2889_amd import FlameSim, native

    w = synth.WORKLOADS[args.workload]
    half = synth.workload_spectrum(w)
    sim = FlameSim(w.n1, w.n2, gamma=w.gamma, theta_pi=w.theta_pi, t0=w.t0, dt=w.dt)
    diag_buf = torch.zeros((max(1, args.steps // max(1, args.diag_every)) + 1, 4), dtype=torch.float64,
                           device=sim.device)
    sim_graph_steps = [0]

    ran = {"graph_replays": 0, "direct_steps": 0, "diagnostics": 0}

    def run_steps(k, time_kernels, count=None):
        """k steps with the diagnostics every diag_every steps (counted from
        the start of this call); `count` (a dict) receives what ran."""
        if time_kernels:
            sim.timing_begin()
        done, d = 0, 0
        gs = sim_graph_steps[0]
        while done < k:
            chunk = min(args.diag_every - (done % args.diag_every), k - done)
            sim.step(chunk)
            if count is not None:
                reps = chunk // gs if gs else 0
                count["graph_replays"] += reps
                count["direct_steps"] += chunk - reps * gs
            done += chunk
            if done % args.diag_every == 0:
                sim.diagnostics(out=diag_buf[d % diag_buf.shape[0]])
                d += 1
                if count is not None:
                    count["diagnostics"] += 1
        return sim.timing_end() if time_kernels else None

    # points per thread of the step kernels chosen by the library's autotuner
    sim.set_spectrum(half)
    if args.pts or args.grid or args.stores:
        if args.grid:
            sim.set_product_grid(w.n1, w.n2, args.grid == "product")
        if args.pts:
            sim.set_points_per_thread(w.n1, w.n2, *args.pts)
        if args.stores:
            sim.set_streaming_stores(w.n1, w.n2, STORE_KINDS[args.stores])
    else:
        # 100 timed steps per trial: with 20 the choice between configurations within
        # 2 % of each other followed the trials' timing noise from box to box
        sim.autotune(steps=100)
    pts = sim.points_per_thread(w.n1, w.n2)
    rows = 3 * w.n1 // 4 if sim.product_grid(w.n1, w.n2) else w.n1
    streaming = sim.streaming_stores(w.n1, w.n2)

    # steps between diagnostics run as one hipGraph replay (a shorter timed
    # region replays graphs of its own length)
    graph_steps = 0 if args.no_graph else min(args.diag_every, max(1, args.steps))
    sim.set_graph_steps(graph_steps)
    sim_graph_steps[0] = graph_steps

    # warm-up from the initial condition (instantiates the graph)
    sim.set_spectrum(half)
    run_steps(max(args.warmup, graph_steps), False)
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()
    # timed region 1: the step as the library runs it (graph replays between diagnostics) -> value
    sim.set_spectrum(half)
    sim.step(0)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    run_steps(args.steps, False, ran)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)

    # timed region 2: the same steps launched directly, every step kernel carrying
    # its own start/stop events -> per-kernel durations for the roofline
    sim.set_graph_steps(0)
    sim_graph_steps[0] = 0
    sim.set_spectrum(half)
    sim.step(0)
    torch.cuda.synchronize()
    kt = run_steps(args.steps, True)
    torch.cuda.synchronize()
    final_diag = diag_buf[0].cpu().tolist()

    nbytes = algorithmic_bytes(w.n1, w.n2, rows)
    per_launch = {k: kt[k][0] / max(1, kt[k][1]) for k in ("row", "col")}
    # The roofline object is the column kernel's: it moves most of the step's
    # bytes (54.5 of 92.2 MB at 2048x4096) and is HBM-bound, while the row kernel
    # is bound by its vector ALU (its own figures follow under roofline_row). The
    # two take about the same time; which is longer changes from box to box.
    dom = "col"
    achieved = nbytes[dom] / (per_launch[dom] * 1e-3) / 1e9
    traffic = measured_traffic(dom, w.name, pts[0] if dom == "col" else pts[1], rows, streaming)
    row_cols = 3 * w.n2 // 4 if pts[1] == 12 else w.n2
    row_flops = row_pass_flops(rows, row_cols)
    row_tflops = row_flops / (per_launch["row"] * 1e-3) / 1e12
    result = {
        "metric": "flame point-steps/s fwd & adjoint, FP32 vs FP64 oracle at 1e-5; % HBM roofline",
        "value": w.points * args.steps / (ms * 1e-3),
        "unit": "point-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "grid": [w.n1, w.n2], "dt": w.dt, "t0": w.t0, "gamma": w.gamma,
                   "diagnostics_every": args.diag_every, "ic": f"{w.rule} modes, amp {w.amp}, seed {w.seed}",
                   "points_per_thread": {"col": pts[0], "row": pts[1]}, "product_rows": rows,
                   "product_cols": 3 * w.n2 // 4 if pts[1] == 12 else w.n2,
                   "streaming_stores": streaming, "graph_steps": graph_steps,
                   # what the timed region ran: graph replays of graph_steps steps, steps
                   # launched directly, and diagnostics (due every diagnostics_every steps)
                   "timed_region": dict(ran, steps=args.steps)},
        "roofline": {
            "bound": "hbm",
            "kernel": f"{dom}_kernel",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "bytes_per_launch": nbytes[dom],
            "ms_per_launch": per_launch[dom],
        },
        "roofline_row": {
            "bound": "alu",
            "kernel": "row_kernel",
            "achieved": row_tflops,
            "peak": FP32_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": row_tflops / FP32_VECTOR_PEAK_TFLOPS,
            "frac_of_unpacked_peak": row_tflops / FP32_UNPACKED_PEAK_TFLOPS,
            "flops_per_launch": row_flops,
            "ms_per_launch": per_launch["row"],
            "hbm_GB_s": nbytes["row"] / (per_launch["row"] * 1e-3) / 1e9,
            "hbm_frac": nbytes["row"] / (per_launch["row"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
        },
        "kernels_ms_per_step": {k: kt[k][0] / max(1, args.steps) for k in ("row", "col", "diag")},
        "step_bytes": nbytes["row"] + nbytes["col"],
        "step_hbm_frac": (nbytes["row"] + nbytes["col"]) / (ms / args.steps * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "diagnostics_at_first_checkpoint": final_diag,
    }
    # the same step bytes against a plain device copy measured on this GPU: one of
    # 256 MiB (source and destination exceed the 256 MB Infinity Cache: HBM); one
    # of 48 MiB like the step's working set follows at the end of the run
    copy_gbs = copy_bandwidth(256 << 20)
    step_gbs = (nbytes["row"] + nbytes["col"]) / (ms / args.steps * 1e-3) / 1e9
    result["copy_bandwidth"] = {
        "GB_s": copy_gbs, "bytes": 256 << 20,
        "step_frac": step_gbs / copy_gbs,
        "dominant_kernel_frac": achieved / copy_gbs,
    }

    # The other legs: a refusal by the library (FlameError, raised before any
    # launch) is recorded under the leg's key instead of ending the run, so the
    # line above is never lost to an optional leg.
    def leg(key, fn, *a, **kw):
        try:
            result[key] = fn(*a, **kw)
        except native.FlameError as e:
            result[key] = {"error": str(e)}

    if args.forcing_steps > 0:
        leg("forced", forced_leg, sim, w, half, args.forcing_steps, graph_steps, run_steps, ms / args.steps, rows)

    if args.heun_steps > 0:
        leg("heun", heun_leg, w, half, args.heun_steps, graph_steps, args.diag_every, ms / args.steps)

    if not args.no_long_run:
        leg("long_run", long_run_leg, t_end=args.long_run_t_end)

    if args.circle_steps > 0:
        rec = circle_record()
        leg("circles", circle_leg, steps=args.circle_steps,
            valu_per_wave_step=rec.get("valu_per_wave_step") if rec else None)
    if not args.no_circle_long_run:
        leg("circle_long_run", circle_long_run_leg)

    if args.adjoint_steps > 0:
        leg("adjoint", adjoint_leg, args.adjoint_steps, 50)
    if args.ensemble_steps > 0:
        leg("ensemble", ensemble_leg, args.ensemble_steps, 50)

    if not args.no_cpu:
        base, nref, ref = cpu_oracle_baseline(w, half, args.cpu_seconds)
        result["cpu_baseline"] = base
        result["cpu_baseline_all_cores"] = cpu_oracle_baseline(w, half, args.cpu_seconds, workers=host_cores())[0]
        sim.set_spectrum(half)
        sim.step(nref)
        got = sim.spectrum().cpu().numpy().astype(np.complex128)
        wgt = np.full(ref.shape, 2.0)
        wgt[:, 0] = 1.0
        err = float(np.sqrt((wgt * np.abs(got - ref) ** 2).sum() / (wgt * np.abs(ref) ** 2).sum()))
        result["parity"] = {"rel_l2_vs_oracle": err, "steps": nref, "tolerance": 1e-5}
    else:
        result["cpu_baseline"] = None
    # A copy of 48 MiB, like the step's working set (W, Q and the state, ~46 MB at
    # 2048x4096), which stays resident in the Infinity Cache from kernel to
    # kernel. Measured last: its torch graph capture slows later hipGraph
    # replays of the library in the same process (by ~13 % on the ensemble).
    resident_gbs = copy_sweep(mib=(48,))["48"]
    result["copy_bandwidth"].update({
        "resident_GB_s": resident_gbs, "resident_bytes": 48 << 20,
        "step_frac_resident": step_gbs / resident_gbs,
        "dominant_kernel_frac_resident": achieved / resident_gbs,
    })
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
