#!/usr/bin/env python3
"""Benchmark of the HWENO shallow-water hot path on one MI355X.

Workload (default): the 2D dam break on a 4096 x 4096 grid, 9 FP64 fields (eta, m, w and their
x- and y-derivatives), reflective walls, a seeded bottom of 4 Gaussian bumps, eta = 10 left of a
random-phase sinusoidal interface near x = 0.5 and 5 right of it. A step is one SSP-RK3 step:
three fused stage kernels (right-hand side + derivative limiter + Runge-Kutta combination +
max-reduction of the next Lax-Friedrichs speeds) and a one-thread prologue (dt). Inputs are
resident in HBM before the timed region.

value = cell right-hand sides per second over the timed steps (3 per node per step).
roofline = the fused stage kernel against the FP64 vector peak, with the algorithmic flops per
node counted by the oracle (right-hand side + limiter) plus the Runge-Kutta combination; its
duration comes from HIP events around every stage launch inside the timed region.
cpu_baseline = the oracle (plain C++ FP64, OpenMP over rows) timed on this host on a bounded
sample: --cpu-steps SSP-RK3 steps of the same 4096^2 state.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "2D HWENO RHS cell-updates/s FP64 (% roofline); batched & adjoint vs plain"
PEAK_FP64 = 78.6e12   # FP64 vector FLOP/s (FMA = 2), MI355X
PEAK_FP32 = 157.3e12  # FP32 vector FLOP/s (FMA = 2), MI355X
PEAK_HBM = 8.0e12     # B/s
RK_FLOPS = (18 + 45 + 45) / 3.0   # per node per stage: U + dt R; (3a + b)/4; (a + 2b)/3, 9 fields
SPEED_FLOPS = 8                   # |u| + c, |v| + c per node (h, 1/h, 2 products, sqrt, 2 adds)
STAGE_BYTES = (27 * 8 + 30 * 8 + 30 * 8) / 3.0  # per node: stage 1 reads 12 writes 15; 2, 3 read 21 write 9
RHS_BYTES = 21 * 8                               # bare right-hand side: read 12, write 9


STAGE_KERNELS = tuple(f"_ZN3swe7k_stageIdLi2ELi{m}EEEvNS_5KArgsIT_EE" for m in range(4))


def _elf_sections(b, base=0):
    """(name, addr, offset, size, link) of each section of the ELF64 image at b[base:]."""
    import struct

    shoff = struct.unpack_from("<Q", b, base + 0x28)[0]
    shentsize, shnum, shstrndx = struct.unpack_from("<HHH", b, base + 0x3A)
    raw = [struct.unpack_from("<IIQQQQII", b, base + shoff + i * shentsize) for i in range(shnum)]
    names = base + raw[shstrndx][4]
    return [(b[names + r[0]:b.index(b"\0", names + r[0])].decode(), r[3], base + r[4], r[5], r[6]) for r in raw]


def device_code_sha(lib=None):
    """sha256[:16] of the machine code and kernel descriptors (without their layout-dependent
    entry offset) of the 2D FP64 stage kernels (k_stage<double, 2, 0..3>) in the gfx950 code
    object of the built solver library. Host code and other kernels leave it unchanged; any change
    to these kernels, to the routines they inline or to their compile flags changes it. None if
    it cannot be read."""
    import struct

    path = lib or os.path.join(ROOT, "paper_2208_01260_amd", "libswe_hweno.so")
    try:
        with open(path, "rb") as f:
            b = f.read()
        fat = next(s for s in _elf_sections(b) if s[0] == ".hip_fatbin")
        fb = b[fat[2]:fat[2] + fat[3]]
        magic = b"__CLANG_OFFLOAD_BUNDLE__"
        if not fb.startswith(magic):
            return None
        pos, co = len(magic) + 8, None
        for _ in range(struct.unpack_from("<Q", fb, len(magic))[0]):
            off, size, tlen = struct.unpack_from("<QQQ", fb, pos)
            triple = fb[pos + 24:pos + 24 + tlen].decode()
            pos += 24 + tlen
            if triple.endswith("gfx950"):
                co = fb[off:off + size]
        if co is None:
            return None
        secs = _elf_sections(co)
        symtab = next(s for s in secs if s[0] == ".symtab")
        strtab = secs[symtab[4]][2]
        want = set(STAGE_KERNELS) | {k + ".kd" for k in STAGE_KERNELS}
        found = {}
        for i in range(symtab[3] // 24):
            nm, _info, _other, shndx, value, size = struct.unpack_from("<IBBHQQ", co, symtab[2] + 24 * i)
            name = co[strtab + nm:co.index(b"\0", strtab + nm)].decode()
            if name in want:
                sec = secs[shndx]
                body = bytearray(co[sec[2] + value - sec[1]:sec[2] + value - sec[1] + size])
                if name.endswith(".kd"):
                    body[16:24] = bytes(8)  # kernel_code_entry_byte_offset: moves with the layout
                found[name] = bytes(body)
        if set(found) != want:
            return None
        h = hashlib.sha256()
        for name in sorted(found):
            h.update(name.encode() + b"\0" + found[name])
        return h.hexdigest()[:16]
    except (OSError, StopIteration, struct.error, UnicodeDecodeError, ValueError, IndexError):
        return None


def measured_traffic(workload):
    """HBM bytes per stage launch from the committed rocprofv3 PMC summary, if it was taken on
    the device code that runs now (else None)."""
    path = os.path.join(ROOT, "profiles", "stage_kernel_traffic.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    sha = device_code_sha()
    if sha is None or d.get("device_code_sha") != sha or d.get("workload") != workload:
        return None
    return d.get("hbm_bytes_per_launch")


def measured_counters(workload):
    """FP64 operations per node of each stage kernel as the GPU executes them (rocprofv3 PMC
    SQ_INSTS_VALU_FLOPS_FP64 ... counts, an FMA counting 2), from the committed summary, if it was
    taken on the device code that runs now (else None)."""
    path = os.path.join(ROOT, "profiles", "stage_kernel_counters.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    sha = device_code_sha()
    if sha is None or d.get("device_code_sha") != sha or d.get("workload") != workload:
        return None
    return d


def device_ceilings(torch, dev):
    """What this device sustains, measured live beside the published peaks: a dense FP64 FMA
    stream (eight independent chains per lane) at 1, 2, 4 and 8 wavefronts per SIMD, about 0.3 s
    of back-to-back launches each, and a device-to-device copy of 2 GiB (bytes read + written per
    second). The stage kernel runs one wavefront per SIMD."""
    from paper_2208_01260_amd.calib import fp64_fma_ceiling

    by_waves = {}
    for w in (1, 2, 4, 8):
        try:
            by_waves[w] = fp64_fma_ceiling(w, 0.3)
        except RuntimeError as e:  # a placement the device cannot make (LDS per block)
            print(f"[bench] FMA stream at {w} wavefronts per SIMD: {e}", file=sys.stderr, flush=True)
    n = (1 << 30) // 8
    a = torch.empty(n, dtype=torch.float64, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 2.0 * a.numel() * 8 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    best = max(v[0] for v in by_waves.values())
    print("[bench] device ceilings: FP64 FMA stream " +
          ", ".join(f"{v[0]:.1f} TFLOP/s at {v[1]:.0f} MHz ({w} wave/SIMD)" for w, v in by_waves.items()) +
          f"; copy {copy_gbs:.0f} GB/s", file=sys.stderr, flush=True)
    return {"fp64_fma_stream_tflops": best, "fp64_fma_stream_frac_of_peak": best * 1e12 / PEAK_FP64,
            "fp64_fma_stream_by_waves_per_simd": {str(w): {"tflops": v[0], "shader_mhz": v[1]}
                                                  for w, v in by_waves.items()},
            "copy_GBs": copy_gbs, "copy_frac_of_hbm_peak": copy_gbs / 8000.0}


def _sysfs_board():
    """The first GPU's board power (hwmon, microwatts) and current shader-clock level files."""
    import glob

    pw = sorted(glob.glob("/sys/class/drm/card*/device/hwmon/hwmon*/power1_average") +
                glob.glob("/sys/class/drm/card*/device/hwmon/hwmon*/power1_input"))
    clk = sorted(glob.glob("/sys/class/drm/card*/device/pp_dpm_sclk"))
    return (pw[0] if pw else None), (clk[0] if clk else None)


def board_state(torch, s, st, seconds=2.0):
    """Board power and shader clock while the fused stage kernels run back to back (graph replays
    of 20 steps for about `seconds`), sampled from sysfs every 50 ms, beside the idle board just
    before. The MI355X's FP64 peak assumes its 2.4 GHz maximum shader clock; a kernel that holds
    the board at its power limit runs at a lower clock."""
    import re
    import statistics
    import threading

    pw, clk = _sysfs_board()
    if pw is None and clk is None:
        return None
    samples, phase, stop = [], ["idle"], [False]

    def read():
        rec = {"phase": phase[0]}
        try:
            rec["w"] = int(open(pw).read()) / 1e6 if pw else None
        except (OSError, ValueError):
            rec["w"] = None
        try:
            cur = [l for l in open(clk).read().splitlines() if l.rstrip().endswith("*")] if clk else []
            m = re.search(r"(\d+)\s*Mhz", cur[0], re.I) if cur else None
            rec["mhz"] = int(m.group(1)) if m else None
        except OSError:
            rec["mhz"] = None
        return rec

    def loop():
        while not stop[0]:
            samples.append(read())
            time.sleep(0.05)

    th = threading.Thread(target=loop, daemon=True)
    th.start()
    time.sleep(0.5)
    phase[0] = "stage"
    t0, steps = time.perf_counter(), 0
    while time.perf_counter() - t0 < seconds:
        s.run(st, nsteps=20)
        torch.cuda.synchronize()
        steps += 20
    ms_per_step = (time.perf_counter() - t0) * 1e3 / steps
    stop[0] = True
    th.join()

    def med(ph, key):
        v = [r[key] for r in samples if r["phase"] == ph and r.get(key) is not None]
        if ph == "stage":
            v = v[4:]  # the first 200 ms: power and clock still settling
        return statistics.median(v) if v else None

    out = {"source": {"power": pw, "clock": clk}, "stage_steps": steps, "stage_ms_per_step": ms_per_step,
           "idle_board_w": med("idle", "w"), "stage_board_w": med("stage", "w"),
           "idle_shader_mhz": med("idle", "mhz"), "stage_shader_mhz": med("stage", "mhz"),
           "samples": len(samples)}
    print(f"[bench] board while the stage kernels run: {out['stage_board_w']} W at {out['stage_shader_mhz']} MHz "
          f"(idle {out['idle_board_w']} W)", file=sys.stderr, flush=True)
    return out


def flop_counts():
    """Algorithmic flops per node (right-hand side, limiter), counted by the oracle's
    operation-counting scalar and stored by tests/golden/make_flop_counts.py."""
    d = json.load(open(os.path.join(ROOT, "tests", "golden", "flop_counts.json")))
    return d["rhs_flops_per_node"], d["limiter_flops_per_node"]


def cpu_baseline(pr, steps):
    """The oracle on this host: `steps` SSP-RK3 steps of the same workload state."""
    import numpy as np

    import oracle

    oracle.build()
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
    oracle.set_threads(threads)
    p = oracle.params_of(pr)
    state = pr.state
    t0 = time.perf_counter()
    for _ in range(steps):
        state, _dt = oracle.step(p, state, pr.b, pr.bx, pr.by)
    dt = time.perf_counter() - t0
    used = oracle.get_threads()
    # the same step on one thread, on a 1024 x 1024 window of the state (reflective walls at its edges)
    import copy
    w = min(1024, pr.nx, pr.ny)
    sub = copy.copy(pr)
    sl = (slice(0, w), slice(0, w))
    sub.state = np.ascontiguousarray(pr.state[(slice(None),) + sl])
    sub.b, sub.bx, sub.by = [np.ascontiguousarray(a[sl]) for a in (pr.b, pr.bx, pr.by)]
    sub.nx = sub.ny = w
    x0, _, y0, _ = pr.domain
    ps = oracle.params_of(sub, domain=(x0, x0 + w * pr.dx, y0, y0 + w * pr.dy))
    oracle.set_threads(1)
    t0 = time.perf_counter()
    oracle.step(ps, sub.state, sub.b, sub.bx, sub.by)
    dt1 = time.perf_counter() - t0
    oracle.set_threads(threads)
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), model)
    except OSError:
        pass
    return {"value": 3.0 * pr.cells * steps / dt, "unit": "cell-RHS/s", "cores": used,
            "kind": "oracle", "host_cpu": model, "host_logical_cpus": os.cpu_count(),
            "sample": f"{steps} SSP-RK3 step(s) (3 right-hand sides, limiter, update each) of the same "
                      f"{pr.nx}x{pr.ny} dam-break state, {dt:.1f} s wall on {used} threads",
            "single_thread_value": 3.0 * w * w / dt1,
            "single_thread_sample": f"1 step of a {w}x{w} window of the same state on 1 thread, {dt1:.1f} s wall"}


def single_precision(args, torch, pr, f_rhs):
    """The FP32 variant on the same workload: the bare right-hand side kernel (alpha given) and
    graph-replayed steps."""
    from paper_2208_01260_amd.solver import Solver

    cells = pr.cells
    st0 = torch.from_numpy(pr.state).to(device="cuda:0", dtype=torch.float32).contiguous()
    with Solver.from_problem(pr, dtype=torch.float32) as s:
        st = st0.clone()
        ax, ay = s.alpha(st)
        out = torch.empty_like(st)
        s.set_timing(True)
        for _ in range(args.warmup):
            s.rhs(st, out, alpha=(ax, ay))
        s.set_timing(True)
        for _ in range(args.steps):
            s.rhs(st, out, alpha=(ax, ay))
        tim = s.get_timing()
        rhs_ms = tim["rhs"][0] / tim["rhs"][1]
        s.set_timing(False)
        s.run(st, nsteps=args.warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.run(st, nsteps=args.steps)
        torch.cuda.synchronize()
        step_ms = (time.perf_counter() - t0) * 1e3 / args.steps
    print(f"[bench] fp32: rhs {rhs_ms:.3f} ms, step {step_ms:.3f} ms", file=sys.stderr, flush=True)
    return {"rhs_avg_launch_ms": rhs_ms, "rhs_cell_updates_per_s": cells / (rhs_ms * 1e-3),
            "rhs_tflops": f_rhs * cells / (rhs_ms * 1e-3) / 1e12,
            "rhs_frac_fp32_peak": f_rhs * cells / (rhs_ms * 1e-3) / PEAK_FP32,
            "ms_per_step": step_ms, "cell_rhs_per_s": 3.0 * cells / (step_ms * 1e-3)}


def adjoint_cost(args, torch):
    """Reverse mode against the plain forward run of the same steps (fixed dt, frozen speeds):
    swe_hweno_run_vjp (its own checkpointed forward, recomputation and reverse), and the autograd
    split: swe_hweno_run_checkpointed (forward keeping checkpoints) and
    swe_hweno_run_vjp_checkpointed (recomputation and reverse). On the adjoint workload (256^2,
    100 steps, checkpoint every 10) and on the same recipe at 2048^2 (20 steps, checkpoint every
    10), where a stage fills the GPU."""
    from paper_2208_01260_amd import inputs
    from paper_2208_01260_amd.solver import FIXED_ALPHA, FIXED_DT, Solver

    def one(n, nsteps, ck, reps):
        pr = inputs.c5_adjoint(n)
        st0 = torch.from_numpy(pr.state).to("cuda:0").contiguous()
        with Solver.from_problem(pr) as s:
            ax, ay = s.alpha(st0)
        al = (1.1 * ax, 1.1 * ay)
        dt = 0.6 / (al[0] / pr.dx + al[1] / pr.dy)

        def timed(fn):
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            return (time.perf_counter() - t0) / reps * 1e3

        with Solver.from_problem(pr, flags=FIXED_DT | FIXED_ALPHA, fixed_dt=dt, alpha=al) as s:
            st = st0.clone()
            sbar = torch.randn_like(st0)

            def fwd():
                st.copy_(st0)
                s.run(st, nsteps=nsteps)

            def fwd_ck():
                st.copy_(st0)
                s.run_checkpointed(st, nsteps, ck)

            fwd_ms = timed(fwd)
            vjp_ms = timed(lambda: s.run_vjp(st0, nsteps, sbar, ck))
            fwd_ck_ms = timed(fwd_ck)
            bwd_ms = timed(lambda: s.run_vjp_checkpointed(nsteps, sbar, ck))
        print(f"[bench] adjoint {n}^2 x {nsteps}: forward {fwd_ms:.2f} ms, run_vjp {vjp_ms:.2f} ms "
              f"({vjp_ms / fwd_ms:.2f}x); checkpointed forward {fwd_ck_ms:.2f} ms, backward {bwd_ms:.2f} ms "
              f"({bwd_ms / fwd_ms:.2f}x)", file=sys.stderr, flush=True)
        return {"workload": f"{n}x{n}, {nsteps} steps, fixed dt, frozen alpha, checkpoint every {ck}",
                "forward_ms": fwd_ms, "run_vjp_ms": vjp_ms, "run_vjp_over_forward": vjp_ms / fwd_ms,
                "checkpointed_forward_ms": fwd_ck_ms, "backward_ms": bwd_ms, "backward_over_forward": bwd_ms / fwd_ms}

    out = one(256, 100, 10, 3)
    if args.adjoint_large > 0:
        out["large"] = one(args.adjoint_large, 20, 10, 2)
    return out


def batched(args, torch):
    """Batched forward solver: `count` independent instances of uneven sizes (64..512 nodes per
    side, seeded bottoms and Gaussian humps, reflective walls), every stage one launch over all
    instances' tiles, against the same instances advanced one plain context after another."""
    from paper_2208_01260_amd import inputs
    from paper_2208_01260_amd.solver import Batch, Solver

    probs = inputs.c4_batch(args.batch_count)
    cells = sum(p.nx * p.ny for p in probs)
    with Batch(probs) as bt:
        rows = bt.autotune()
        bt.run(args.warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bt.run(args.batch_steps)
        torch.cuda.synchronize()
        wall_b = time.perf_counter() - t0
    # plain contexts, one instance after another (graph replay each), on a subset that keeps
    # this leg short; the rate is per cell-step so the subset size does not matter
    sub = probs[: max(1, min(len(probs), args.batch_loop))]
    sub_cells = sum(p.nx * p.ny for p in sub)
    ctxs = [(Solver.from_problem(p), torch.from_numpy(p.state).cuda().contiguous()) for p in sub]
    for s, st in ctxs:
        s.run(st, nsteps=args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s, st in ctxs:
        s.run(st, nsteps=args.batch_steps)
    torch.cuda.synchronize()
    wall_p = time.perf_counter() - t0
    for s, _ in ctxs:
        s.close()
    rate_b = cells * args.batch_steps / wall_b
    rate_p = sub_cells * args.batch_steps / wall_p
    print(f"[bench] batch: {len(probs)} instances, {cells} cells, {rate_b:.3e} cell-steps/s "
          f"(plain loop {rate_p:.3e}, rows {rows})", file=sys.stderr, flush=True)
    return {"instances": len(probs), "cells": cells, "steps": args.batch_steps, "rows_per_wave": rows,
            "ms_per_step": wall_b * 1e3 / args.batch_steps, "cell_steps_per_s": rate_b,
            "cell_rhs_per_s": 3.0 * rate_b, "plain_loop_instances": len(sub),
            "plain_loop_cell_steps_per_s": rate_p, "speedup_vs_plain_loop": rate_b / rate_p}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=4096, help="grid nodes per direction")
    ap.add_argument("--cpu-steps", type=int, default=2, help="oracle sample: steps of the same workload")
    ap.add_argument("--no-cpu", action="store_true", help="skip the cpu_baseline leg")
    ap.add_argument("--no-fp32", action="store_true", help="skip the single-precision leg")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the reverse-mode leg")
    ap.add_argument("--adjoint-large", type=int, default=2048,
                    help="grid of the GPU-filling adjoint measurement (0 skips it)")
    ap.add_argument("--batch-count", type=int, default=256, help="instances of the batched leg (0 skips it)")
    ap.add_argument("--batch-steps", type=int, default=20)
    ap.add_argument("--batch-loop", type=int, default=64, help="instances timed one by one for comparison")
    ap.add_argument("--no-power", action="store_true", help="skip the board power / clock sample")
    ap.add_argument("--no-ceilings", action="store_true",
                    help="skip the measured device ceilings (FP64 FMA stream, device copy)")
    ap.add_argument("--copy-calib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (PMC calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; the solver has no multi-GPU path (asked for --gpus {args.gpus}); "
              "each extra GPU would take a slab of rows with a two-row halo exchange per stage", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2208_01260_amd import _lib, inputs
    from paper_2208_01260_amd.solver import Solver

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    t_gen = time.perf_counter()
    pr = inputs.c3_2d(args.n)
    print(f"[bench] inputs {args.n}x{args.n} generated in {time.perf_counter() - t_gen:.1f} s", file=sys.stderr,
          flush=True)
    workload = f"2D dam break {args.n}x{args.n}, 9 FP64 fields, reflective walls, seeded Gaussian bottom"
    cells = pr.cells
    dev = torch.device("cuda:0")
    state0 = torch.from_numpy(pr.state).to(dev).contiguous()
    st = state0.clone()
    s = Solver.from_problem(pr, device=dev)
    tile = s.tile()
    torch.cuda.synchronize()

    # warm-up (graph path), then the graph path timed for reference
    s.run(st, nsteps=args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.run(st, nsteps=args.steps)
    torch.cuda.synchronize()
    graph_ms = (time.perf_counter() - t0) * 1e3 / args.steps
    print(f"[bench] graph replay: {graph_ms:.3f} ms/step", file=sys.stderr, flush=True)

    # timed region: the same steps with an event pair around every fused stage kernel
    st.copy_(state0)
    s.set_timing(True)
    s.run(st, nsteps=args.warmup)
    s.set_timing(True)  # reset the totals
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    t_sim, k = s.run(st, nsteps=args.steps)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = ev0.elapsed_time(ev1)
    tim = s.get_timing()
    stage_ms = sum(tim[f"stage{i}"][0] for i in (1, 2, 3))
    stage_n = sum(tim[f"stage{i}"][1] for i in (1, 2, 3))
    assert k == args.steps and stage_n == 3 * args.steps, (k, stage_n)
    ms_per_step = wall * 1e3 / args.steps
    value = 3.0 * cells * args.steps / wall
    print(f"[bench] timed: {ms_per_step:.3f} ms/step (events {ev_ms / args.steps:.3f}), stage kernel "
          f"{stage_ms / stage_n:.3f} ms/launch", file=sys.stderr, flush=True)

    # the bare right-hand side kernel (the metric's unit), alpha given
    ax, ay = s.alpha(st)
    out = torch.empty_like(st)
    s.set_timing(True)
    for _ in range(3):
        s.rhs(st, out, alpha=(ax, ay))
    per = []
    for _ in range(max(args.steps, 20)):  # each launch bracketed by its own event pair
        s.set_timing(True)
        s.rhs(st, out, alpha=(ax, ay))
        t_one = s.get_timing()["rhs"]
        per.append(t_one[0] / t_one[1])
    rhs_ms = sum(per) / len(per)
    rhs_median_ms = sorted(per)[len(per) // 2]
    s.set_timing(False)

    f_rhs, f_lim = flop_counts()
    f_stage = f_rhs + f_lim + RK_FLOPS + SPEED_FLOPS
    avg_s = stage_ms / stage_n * 1e-3
    achieved = f_stage * cells / avg_s
    traffic = measured_traffic(workload)
    counters = measured_counters(workload)
    roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64, "traffic": traffic,
            "kernel": "k_stage<2,*> (fused stage: RHS + limiter + RK update + alpha reduction)",
            "flops_per_node": f_stage, "algorithmic_bytes_per_node": STAGE_BYTES,
            "hbm_achieved_GBs": STAGE_BYTES * cells / avg_s / 1e9,
            "avg_launch_ms": avg_s * 1e3}
    if counters is not None:
        # what the GPU executes: the kernel's rearrangements need fewer FP64 operations per node
        # than the oracle's plain count that the headline fraction uses
        fe = counters["stage_fp64_flops_per_node"]
        roof["executed"] = {"fp64_flops_per_node": fe, "tflops": fe * cells / avg_s / 1e12,
                            "frac": fe * cells / avg_s / PEAK_FP64, "source": counters["source"]}
    rhs_kernel = {"avg_launch_ms": rhs_ms, "median_launch_ms": rhs_median_ms, "launches": len(per),
                  "cell_updates_per_s": cells / (rhs_ms * 1e-3),
                  "flops_per_node": f_rhs, "tflops": f_rhs * cells / (rhs_ms * 1e-3) / 1e12,
                  "frac_fp64_peak": f_rhs * cells / (rhs_ms * 1e-3) / PEAK_FP64,
                  "hbm_GBs": RHS_BYTES * cells / (rhs_ms * 1e-3) / 1e9}

    if args.copy_calib:
        # plain streaming kernels of known size for PMC calibration: a fill (writes N bytes) and
        # an elementwise b = a + 1 (reads N bytes, writes N bytes)
        n = args.copy_calib * (1 << 20) // 8
        a = torch.empty(n, dtype=torch.float64, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            torch.add(a, 1.0, out=b)
        torch.cuda.synchronize()

    line = {
        "metric": METRIC, "value": value, "unit": "cell-RHS/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": workload, "nx": args.n, "ny": args.n, "fields": 9, "step": "SSP-RK3 (3 fused stages)",
                   "sim_time_advanced": t_sim},
        "roofline": roof,
        "rhs_kernel": rhs_kernel,
        "graph_replay_ms_per_step": graph_ms,
        "tile": {"cols_per_wave": tile[0], "rows_per_wave": tile[1]},
        "library": {"path": os.path.relpath(_lib.LIB_PATH, ROOT), "source_hash": _lib.check_stamp(_lib.lib()),
                    "stage_code_sha": device_code_sha()},
        "cell_steps_per_s": cells * args.steps / wall,
    }
    if not args.no_power:
        board = board_state(torch, s, st)
        if board is not None:
            line["board"] = board
            if board.get("stage_shader_mhz"):
                # the same kernel time against the peak at the clock the board sustained
                roof["frac_at_sustained_clock"] = achieved / (PEAK_FP64 * board["stage_shader_mhz"] / 2400.0)
    s.close()
    if not args.no_ceilings:
        line["device_ceilings"] = device_ceilings(torch, dev)
        fma = line["device_ceilings"]["fp64_fma_stream_tflops"]
        roof["frac_of_fp64_fma_stream"] = achieved / 1e12 / fma
        rhs_kernel["frac_of_fp64_fma_stream"] = rhs_kernel["tflops"] / fma
    if not args.no_fp32:
        line["fp32"] = single_precision(args, torch, pr, f_rhs)
    if args.batch_count > 0:
        line["batched"] = batched(args, torch)
    if not args.no_adjoint:
        line["adjoint"] = adjoint_cost(args, torch)
    if not args.no_cpu:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(pr, args.cpu_steps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
