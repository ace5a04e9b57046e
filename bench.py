"""Throughput of the split SL-MPP5 Vlasov step on one MI355X.

One step is the nine sweeps of Eq. (5) (half kicks ux,uy,uz; drifts z,y,x;
half kicks ux,uy,uz) over the whole 6D grid.  The default workload is the
throughput shape, 64^3 spatial x 32^3 velocity cells (8.59e9 cells, 34.4 GB
per FP32 copy), with the seeded initial condition and drifting potential of
``paper_2110_15867_amd.inputs``.  Inputs and all fields are resident in HBM
before the timed region.

Prints ONE JSON line: cell-updates/s per full step, the algorithmic HBM rate
of the step against the 8 TB/s peak, a roofline entry for the slowest launch
(HIP events on the launch stream; every launch streams f once in and once
out), each kernel's time per timed step, the same workload with FP16 storage
(speedup against FP32; skipped with --no-fp16 or when --prec is not f32),
companion timings (merged half kicks, fused moments, the step adjoint, 64^3
velocity blocks) and
the FP64 CPU oracle timed on a bounded sample on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E
# The full step should move its algorithmic bytes at this fraction of the HBM
# peak or better.
TARGET_FRAC = 0.70


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def algorithmic_bytes_per_cell(prec: int, nuz: int) -> float:
    """One read and one write of f per sweep (codes, plus scales for FP16/BF16)."""
    if prec == 0:
        return 8.0
    return 2.0 * (2.0 + 4.0 / nuz)


# The sources of the profiled kernels (the kick, the position sweeps, the copy
# kernel that calibrates the counters) and of the host code that launches
# them; the moments, field, adjoint and background files hold none of them.
TRAFFIC_SOURCES = ("capi.hip", "kick.hip", "launch.hpp", "probe.hip", "rows.hpp", "sl_mpp5.hpp",
                   "sweeps.hip", "sweeps_bf16.hip", "sweeps_f16.hip", "sweeps_f32.hip",
                   "sweeps_impl.hpp")


def kernel_source_hash() -> str:
    import hashlib

    h = hashlib.sha256()
    for name in TRAFFIC_SOURCES:
        h.update(name.encode())
        with open(os.path.join(ROOT, "paper_2110_15867_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(prec: int, kernel: str, nu: int, nx: int):
    """HBM bytes per dispatch from the committed rocprofv3 counter summary, if it
    was taken on the current sources of the profiled kernels (else None)."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    data = json.load(open(path)).get({0: "f32", 1: "f16", 2: "bf16"}[prec])
    if not data or data.get("source_sha256") != kernel_source_hash():
        return None
    if kernel == "kick":
        prefix = f"k_kick<{prec}, {nu}, "
    else:
        prefix = f"k_position<{prec}, {1 if kernel == 'z' else 4}, {nx}, "
    hits = [v for k, v in data["bytes_per_dispatch"].items() if k.startswith(prefix)]
    return hits[0] if len(hits) == 1 else None


# MI355X vector ALU issue rate without packed FP32 instructions (the kernels
# are built without them): 256 CUs x 4 SIMDs x 16 lanes per clock x 2.4 GHz
# (each wave64 VALU instruction occupies a SIMD for four clocks).
VALU_PEAK_TLANE_OPS = 256 * 4 * 16 * 2.4e9 / 1e12


def measured_valu(prec: int, kernel: str, nu: int, nx: int):
    """VALU lane-operations per dispatch (SQ_INSTS_VALU x 64) from the committed
    rocprofv3 counter summary, if it was taken on the current sources of the
    profiled kernels (else None)."""
    path = os.path.join(ROOT, "profiles", "valu_counts.json")
    if not os.path.exists(path):
        return None
    data = json.load(open(path)).get({0: "f32", 1: "f16", 2: "bf16"}[prec])
    if not data or data.get("source_sha256") != kernel_source_hash():
        return None
    if kernel == "kick":
        prefix = f"k_kick<{prec}, {nu}, "
    else:
        prefix = f"k_position<{prec}, {1 if kernel == 'z' else 4}, {nx}, "
    hits = [v for k, v in data["lane_ops_per_dispatch"].items() if k.startswith(prefix)]
    return hits[0] if len(hits) == 1 else None


def cpu_baseline(seconds: float = 12.0):
    """FP64 oracle Strang step on the 16^3 x 16^3 workload (same recipe), host cores."""
    import numpy as np

    import oracle
    from paper_2110_15867_amd import inputs

    w = inputs.workload(1)
    g = oracle.Grid.make(w.n, w.nu, w.L, w.umax)
    f = inputs.initial_f(w)
    pot = inputs.potential(w)
    steps, t_used, cpu_used = 0, 0.0, 0.0
    while t_used < seconds and steps < 20:
        gn = inputs.accel_field(w, pot, steps * w.dt)
        gnp1 = inputs.accel_field(w, pot, (steps + 1) * w.dt)
        t0, c0 = time.perf_counter(), time.process_time()
        f = oracle.step(g, f, gn, gnp1, w.dt)
        t_used += time.perf_counter() - t0
        cpu_used += time.process_time() - c0
        steps += 1
    # threads actually busy: CPU time of the process over wall time (numpy's
    # elementwise kernels run on one thread; a threaded BLAS call would add)
    cores = max(1, int(round(cpu_used / t_used)))
    return {
        "value": w.cells * steps / t_used,
        "unit": "cell-updates/s",
        "cores": cores,
        "kind": "oracle",
        "sample": f"FP64 oracle Strang step on 16^3x16^3 cells (same recipe), {steps} steps, "
                  f"{t_used:.1f} s",
    }


def timed_run(V, torch, inputs, w, grid, prec, K, W, dev, stream):
    """K timed steps of one storage form; inputs resident in HBM first."""
    # ---- inputs resident in HBM ----
    f0 = inputs.initial_f32_device(w, dev)
    state = V.encode(grid, prec, f0)
    if prec != V.F32:
        del f0
    pot = inputs.potential(w)
    nfield = W + 2 * K + 1
    fields = [torch.from_numpy(inputs.accel_field(w, pot, n * w.dt)).to(dev)
              for n in range(nfield)]
    out = V.empty_state(grid, prec, dev)
    work_bytes = V.vlasov_step_workspace_bytes(grid, prec)
    work = torch.empty(work_bytes, dtype=torch.uint8, device=dev)
    outflow = torch.zeros(tuple(w.n), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    _log("bench: inputs ready")

    # Each step is the five launches vlasov_step makes -- kick(g_n) [ux, uy,
    # uz fused in LDS], z, y, x, kick(g_np1) -- issued through the public
    # single-launch calls so that HIP events between them time every kernel
    # inside the timed region itself (no synchronisation until the end).  The
    # warmup issues the same calls, so no first-call cost lands in the timed
    # region.
    names = ["kick", "z", "y", "x", "kick"]
    wf = V.empty_state(grid, prec, dev)
    bufs = [state, out, wf]                # input, and the two ping-pong targets

    def five_launches(n, ev=None):
        src, b = bufs[0], 0
        gn, gnp1 = fields[n], fields[n + 1]
        if ev is not None:
            ev[0].record(stream)
        for i, nm in enumerate(names):
            dst = (bufs[1], bufs[2])[b]
            if nm == "kick":
                V.vlasov_kick(grid, prec, V.VBC_OUTFLOW, src.f, src.scale, dst.f, dst.scale,
                              gn if i == 0 else gnp1, 0.5 * w.dt, work, work_bytes, outflow,
                              stream)
            else:
                getattr(V, f"vlasov_advect_{nm}")(grid, prec, src.f, src.scale, dst.f, dst.scale,
                                                  w.dt, stream)
            if ev is not None:
                ev[i + 1].record(stream)
            src = dst
            b ^= 1
        bufs[0], bufs[1] = bufs[1], bufs[0]  # five launches end in bufs[1]

    n = 0
    for _ in range(W):
        five_launches(n)
        n += 1
    torch.cuda.synchronize()
    _log("bench: warmup done")

    # ---- timed region: K whole steps ----
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(len(names) + 1)]
           for _ in range(K)]
    torch.cuda.synchronize()
    t_wall0 = time.perf_counter()
    # A short device spin ahead of the first event lets the host queue the
    # first launches before the GPU reaches them, so the events time kernels,
    # not host launch latency after the synchronisation.  It lies outside the
    # events that time the steps.
    torch.cuda._sleep(int(5e6))
    for k in range(K):
        five_launches(n, evs[k])
        n += 1
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall0
    step_ms = [evs[k][0].elapsed_time(evs[k][len(names)]) for k in range(K)]
    total_ms = evs[0][0].elapsed_time(evs[K - 1][len(names)])
    _log(f"bench: timed {K} steps, {total_ms:.1f} ms (wall {t_wall * 1e3:.1f} ms)")
    per = {k: [] for k in ["kick", "z", "y", "x"]}
    for k in range(K):
        for i, nm in enumerate(names):
            per[nm].append(evs[k][i].elapsed_time(evs[k][i + 1]))
    del wf, bufs, state, out, work, fields, outflow
    torch.cuda.empty_cache()
    return {"total_ms": total_ms, "step_ms": step_ms, "per": per, "t_wall": t_wall}


def per_step(per, name, K):
    """Event times of one kernel, one value per timed step (kicks averaged)."""
    v = per[name]
    if len(v) == K:
        return v
    m = len(v) // K
    return [statistics.mean(v[k * m:(k + 1) * m]) for k in range(K)]


def companion_run(V, torch, inputs, w, grid, prec, K, dev, stream):
    """Two other forms of the same work, for comparison (not the headline):
    K steps through vlasov_steps, whose half kicks between steps run as one
    kick (it rounds differently from K single steps), and one step with the
    moments of its result fused into the last kick, against a step followed by
    a moments pass."""
    f0 = inputs.initial_f32_device(w, dev)
    state = V.encode(grid, prec, f0)
    if prec != V.F32:
        del f0
    pot = inputs.potential(w)
    fields = torch.stack([torch.from_numpy(inputs.accel_field(w, pot, k * w.dt))
                          for k in range(K + 1)]).to(dev)
    out = V.empty_state(grid, prec, dev)
    nb = V.vlasov_steps_workspace_bytes(grid, prec)
    work = torch.empty(nb, dtype=torch.uint8, device=dev)
    rho = torch.empty(tuple(w.n), dtype=torch.float64, device=dev)
    um = torch.empty((3,) + tuple(w.n), dtype=torch.float64, device=dev)

    def timed(fn, reps=2):
        fn()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record(stream)
        for _ in range(reps):
            fn()
        ev[1].record(stream)
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1]) / reps

    def merged():
        V.vlasov_steps(grid, prec, V.VBC_OUTFLOW, state.f, state.scale, out.f, out.scale, fields,
                       K, w.dt, None, work, nb, None, stream)

    def step():
        V.vlasov_step(grid, prec, V.VBC_OUTFLOW, state.f, state.scale, out.f, out.scale,
                      fields[0], fields[1], w.dt, 1.0, work, nb, None, stream)

    def step_mom():
        V.vlasov_step_moments(grid, prec, V.VBC_OUTFLOW, state.f, state.scale, out.f,
                              out.scale, fields[0], fields[1], w.dt, 1.0, work, nb, None, rho,
                              um, stream)

    def mom():
        V.vlasov_moments(grid, prec, out.f, out.scale, rho, um, None, stream)

    sig = torch.empty((6,) + tuple(w.n), dtype=torch.float64, device=dev)

    def disp():
        V.vlasov_dispersion(grid, prec, out.f, out.scale, rho, um, sig, stream)

    ms_merged = timed(merged, reps=1) / K
    ms_step, ms_step_mom, ms_mom = timed(step), timed(step_mom), timed(mom)
    ms_disp = timed(disp)
    del state, out, work, fields, rho, um, sig
    torch.cuda.empty_cache()
    return {
        "merged_half_kicks": {
            "value": w.cells / (ms_merged * 1e-3),
            "unit": "cell-updates/s",
            "ms_per_step": ms_merged,
            "steps": K,
            "speedup_vs_single_step_calls": ms_step / ms_merged,
            "form": "vlasov_steps: the two half kicks between steps run as one kick "
                    "(4 passes per step instead of 5); not Eq. (5) step by step",
        },
        "fused_moments": {
            "step_ms": ms_step,
            "step_with_fused_moments_ms": ms_step_mom,
            "separate_moments_pass_ms": ms_mom,
            "dispersion_tensor_pass_ms": ms_disp,
            "dispersion_tensor_pass_GBps": (V.vlasov_f_bytes(grid, prec)
                                            + V.vlasov_scale_bytes(grid, prec)) / (ms_disp * 1e6),
        },
    }


def velocity64_companion(V, torch, inputs, dev, stream, reps=3):
    """vlasov_step (FP32) with 64^3 velocity blocks: the throughput workload's
    recipe on 32^3 x 64^3 cells (as many cells as the headline grid).  A
    64^3 block does not fit a work-group's LDS: each kick runs ux as a
    launch of its own and uy, uz fused on slabs of eight u_x rows, so a step
    is seven passes over f (2 + 3 + 2), each reading and writing 8 B per
    cell."""
    w = inputs.scaled(inputs.workload(3), (32, 32, 32), (64, 64, 64))
    grid = V.make_grid(w.n, w.nu, w.L, w.umax)
    state = V.State(grid, V.F32, inputs.initial_f32_device(w, dev))
    pot = inputs.potential(w)
    gn = torch.from_numpy(inputs.accel_field(w, pot, 0.0)).to(dev)
    gnp1 = torch.from_numpy(inputs.accel_field(w, pot, w.dt)).to(dev)
    out = V.empty_state(grid, V.F32, dev)
    nb = V.vlasov_step_workspace_bytes(grid, V.F32)
    work = torch.empty(nb, dtype=torch.uint8, device=dev)

    def step():
        V.vlasov_step(grid, V.F32, V.VBC_OUTFLOW, state.f, None, out.f, None, gn, gnp1, w.dt,
                      1.0, work, nb, None, stream)

    step()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record(stream)
    for _ in range(reps):
        step()
    ev[1].record(stream)
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / reps
    bytes_step = 7 * 8 * w.cells
    del state, out, work
    torch.cuda.empty_cache()
    return {
        "workload": w.name,
        "value": w.cells / (ms * 1e-3),
        "unit": "cell-updates/s",
        "ms_per_step": ms,
        "passes_per_step": 7,
        "hbm_tbps_algorithmic": bytes_step / (ms * 1e-3) / 1e12,
    }


def adjoint_companion(V, torch, inputs, dev, stream, reps=3):
    """vlasov_step_adj on the differentiation workload (32^3 x 16^3, FP32): the
    eight forward stages recomputed from f, then the nine transposed sweeps.
    Algorithmic bytes per cell: 8 forward sweeps x 8 B + 9 adjoint sweeps x
    12 B (read the stage and the incoming adjoint, write the outgoing one)."""
    w = inputs.workload(5)
    grid = V.make_grid(w.n, w.nu, w.L, w.umax)
    f = inputs.initial_f32_device(w, dev)
    pot = inputs.potential(w)
    gn = torch.from_numpy(inputs.accel_field(w, pot, 0.0)).to(dev)
    gnp1 = torch.from_numpy(inputs.accel_field(w, pot, w.dt)).to(dev)
    lam = torch.ones_like(f)
    lam_in = torch.empty_like(f)
    lgn = torch.zeros_like(gn)
    lgnp1 = torch.zeros_like(gn)
    nb = V.vlasov_step_adj_workspace_bytes(grid)
    work = torch.empty(nb, dtype=torch.uint8, device=dev)
    fwd_out = torch.empty_like(f)
    fwd_nb = V.vlasov_step_workspace_bytes(grid, V.F32)
    fwd_work = torch.empty(fwd_nb, dtype=torch.uint8, device=dev)

    def adj():
        V.vlasov_step_adj(grid, V.VBC_OUTFLOW, f, gn, gnp1, w.dt, 1.0, lam, lam_in, lgn, lgnp1,
                          work, nb, stream)

    def fwd():
        V.vlasov_step(grid, V.F32, V.VBC_OUTFLOW, f, None, fwd_out, None, gn, gnp1, w.dt, 1.0,
                      fwd_work, fwd_nb, None, stream)

    def timed(fn):
        fn()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record(stream)
        for _ in range(reps):
            fn()
        ev[1].record(stream)
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1]) / reps

    ms_adj, ms_fwd = timed(adj), timed(fwd)
    bytes_adj = (8 * 8 + 9 * 12) * w.cells
    del f, lam, lam_in, work, fwd_out, fwd_work
    torch.cuda.empty_cache()
    return {
        "workload": w.name,
        "step_adj_ms": ms_adj,
        "step_ms": ms_fwd,
        "adj_over_step": ms_adj / ms_fwd,
        "bytes_per_step_adj": bytes_adj,
        "hbm_tbps_algorithmic": bytes_adj / (ms_adj * 1e-3) / 1e12,
        "frac": bytes_adj / (ms_adj * 1e-3) / 1e9 / HBM_PEAK_GBS,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--prec", default="f32", choices=["f32", "f16", "bf16"])
    ap.add_argument("--workload", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp16", action="store_true",
                    help="skip the FP16-storage companion run of an FP32 bench")
    ap.add_argument("--no-companions", action="store_true",
                    help="skip the merged-kick and fused-moments companion timings")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the sweeps shard along space across GPUs "
              "(design only, not built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2110_15867_amd import inputs
    from paper_2110_15867_amd import vlasov as V

    prec = {"f32": V.F32, "f16": V.F16, "bf16": V.BF16}[args.prec]
    w = inputs.workload(args.workload)
    grid = V.make_grid(w.n, w.nu, w.L, w.umax)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    K, W = args.steps, args.warmup
    _log(f"bench: {w.name}, {w.cells:.3e} cells, prec {args.prec}, warmup {W}, steps {K}")

    # ---- HBM copy probe: the practical ceiling of a streaming kernel ----
    probe_bytes = 8 << 30
    a_buf = torch.empty(probe_bytes, dtype=torch.uint8, device=dev)
    b_buf = torch.empty(probe_bytes, dtype=torch.uint8, device=dev)
    a_buf.fill_(1)
    V.vlasov_stream_copy(a_buf, b_buf, probe_bytes, stream)
    pe = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    pe[0].record(stream)
    for _ in range(5):
        V.vlasov_stream_copy(a_buf, b_buf, probe_bytes, stream)
    pe[1].record(stream)
    torch.cuda.synchronize()
    copy_gbs = 5 * 2 * probe_bytes / (pe[0].elapsed_time(pe[1]) * 1e-3) / 1e9
    del a_buf, b_buf
    _log(f"bench: copy probe {copy_gbs:.0f} GB/s (read + write)")
    # the vector-ALU ceiling: independent FP32 chains over 2^20 threads
    vbuf = torch.empty(1 << 20, dtype=torch.float32, device=dev)
    V.vlasov_valu_probe(vbuf, 200, stream)
    ve = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ve[0].record(stream)
    ops = 0.0
    for _ in range(3):
        ops += V.vlasov_valu_probe(vbuf, 2000, stream)
    ve[1].record(stream)
    torch.cuda.synchronize()
    valu_probe = ops / (ve[0].elapsed_time(ve[1]) * 1e-3) / 1e12
    del vbuf
    _log(f"bench: VALU probe {valu_probe:.1f} Tlane-op/s")

    r = timed_run(V, torch, inputs, w, grid, prec, K, W, dev, stream)
    total_ms, step_ms, per = r["total_ms"], r["step_ms"], r["per"]
    avg = {k: statistics.mean(v) for k, v in per.items()}
    dominant = max(avg, key=avg.get)
    bpc = algorithmic_bytes_per_cell(prec, w.nu[2])
    launch_bytes = bpc * w.cells
    achieved_gbs = launch_bytes / (avg[dominant] * 1e-3) / 1e9
    traffic = measured_traffic(prec, dominant, w.nu[0], w.n[0])
    # Every launch streams f once in and once out (HBM), and evaluates the flux
    # of every interface (vector ALU).  Both are reported for the slowest
    # launch; the one it is closer to is its bound.  The ALU side counts VALU
    # lane-operations (rocprofv3 SQ_INSTS_VALU x 64 per dispatch, committed
    # summary, guarded by the kernel sources' hash): the early-out of the
    # limiter makes the work per cell data-dependent, so the count, not a
    # fixed formula, is the arithmetic the launch does.
    hbm = {
        "bound": "hbm",
        "kernel": "kick (ux, uy, uz fused)" if dominant == "kick" else f"sweep {dominant}",
        "bytes_per_launch": launch_bytes,
        "achieved": achieved_gbs,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": achieved_gbs / HBM_PEAK_GBS,
        "traffic": traffic,
        "frac_of_copy_probe": achieved_gbs / copy_gbs,
    }
    roofline = hbm
    lane_ops = measured_valu(prec, dominant, w.nu[0], w.n[0])
    if lane_ops is not None:
        valu_t = lane_ops / (avg[dominant] * 1e-3) / 1e12
        alu = {
            "bound": "alu",
            "kernel": hbm["kernel"],
            "lane_ops_per_launch": lane_ops,
            "achieved": valu_t,
            "peak": VALU_PEAK_TLANE_OPS,
            "unit": "Tlane-op/s",
            "frac": valu_t / VALU_PEAK_TLANE_OPS,
            "traffic": traffic,
            "frac_of_valu_probe": valu_t / valu_probe,
        }
        if alu["frac"] > hbm["frac"]:
            roofline = dict(alu, hbm={k: v for k, v in hbm.items() if k not in ("bound", "kernel")})
        else:
            roofline = dict(hbm, alu={k: v for k, v in alu.items() if k not in ("bound", "kernel")})
    _log("bench: per-kernel ms " + json.dumps({k: round(v, 3) for k, v in avg.items()}))
    for nm in per:
        _log(f"bench: {nm} ms per step " + " ".join(f"{x:.2f}" for x in per_step(per, nm, K)))

    value = w.cells * K / (total_ms * 1e-3)
    step_bytes = 5 * launch_bytes              # two fused kicks and three drifts
    step_frac = step_bytes / (total_ms / K * 1e-3) / 1e9 / HBM_PEAK_GBS
    res = {
        "metric": "6D phase-space cell-updates/sec per full step",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": total_ms / K,
        "median_ms_per_step": statistics.median(step_ms),
        "min_ms_per_step": min(step_ms),
        "max_ms_per_step": max(step_ms),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {V.F32: "f32", V.F16: "f16 storage, f32 math",
                  V.BF16: "bf16 storage, f32 math"}[prec],
        "data": "synthetic (seeded Fermi-Dirac-like f0 with random density modes, "
                "drifting 4-mode potential)",
        "config": {"workload": w.name, "nx": list(w.n), "nu": list(w.nu), "L": list(w.L),
                   "dt": w.dt, "sweeps_per_step": 9, "launches_per_step": 5,
                   "storage": args.prec},
        # the bytes the five launches of a step must move (one read and one
        # write of f each), over the step time
        "hbm_tbps_algorithmic": step_bytes / (total_ms / K * 1e-3) / 1e12,
        "step_hbm_frac": step_frac,
        "step_hbm_target_frac": TARGET_FRAC,
        "step_hbm_gap_to_target": TARGET_FRAC - step_frac,
        "kernel_ms": {k: round(v, 4) for k, v in avg.items()},
        # per timed step: each kernel's event time (the kick entry is the mean
        # of the step's two kicks), to tell a trend over the run from noise
        "kernel_ms_per_step": {k: [round(x, 3) for x in per_step(per, k, K)]
                               for k in per},
        "copy_probe_gbs": copy_gbs,
        "valu_probe_tlane_ops": valu_probe,
        "roofline": roofline,
    }
    if args.prec == "f32" and not args.no_fp16:
        # the FP16-storage form of the same workload, for the FP16 vs FP32
        # comparison (its error against the FP64 oracle is a GPU test)
        r16 = timed_run(V, torch, inputs, w, grid, V.F16, K, W, dev, stream)
        avg16 = {k: statistics.mean(v) for k, v in r16["per"].items()}
        ms16 = r16["total_ms"] / K
        bytes16 = 5 * algorithmic_bytes_per_cell(V.F16, w.nu[2]) * w.cells
        res["fp16_storage"] = {
            "value": w.cells * K / (r16["total_ms"] * 1e-3),
            "ms_per_step": ms16,
            "median_ms_per_step": statistics.median(r16["step_ms"]),
            "speedup_vs_f32": (total_ms / K) / ms16,
            "kernel_ms": {k: round(v, 4) for k, v in avg16.items()},
            "hbm_tbps_algorithmic": bytes16 / (ms16 * 1e-3) / 1e12,
        }
        _log("bench: fp16 per-kernel ms " + json.dumps({k: round(v, 3) for k, v in avg16.items()}))
    if not args.no_companions:
        _log("bench: companion timings (merged half kicks, fused moments)")
        res["companions"] = companion_run(V, torch, inputs, w, grid, prec, K, dev, stream)
        _log("bench: companion timing (step adjoint)")
        res["companions"]["step_adjoint"] = adjoint_companion(V, torch, inputs, dev, stream)
        _log("bench: companion timing (64^3 velocity blocks)")
        res["companions"]["velocity_64"] = velocity64_companion(V, torch, inputs, dev, stream)
    if not args.no_cpu_baseline:
        _log("bench: timing the CPU oracle")
        res["cpu_baseline"] = cpu_baseline()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
