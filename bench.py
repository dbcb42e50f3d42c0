#!/usr/bin/env python3
"""Benchmark of the spectral-element Poisson hot path on one MI355X.

Workload (synthetic, seeded): the 32x32x32 brick of E = 32768 hexahedra on
the unit cube at N = 10 GLL nodes per direction, deformed by
x = X + 0.05 sin(2 pi X) sin(2 pi Y) sin(2 pi Z) (likewise y, z), so every
node carries the full six geometric factors in FP64; u ~ U[-1, 1] (seed 0).

One timed step is one application of the matrix-free operator
w_e = D^T G_e D u_e to every element (the paper's AX kernel, Section II-B,
Listing 1), with u, G, D and w resident in HBM.  The value is AX GFLOP/s
counted with the paper's 12N + 11 flops per node (203 per node at 16 nodes
per direction, Section III).  The same run also measures, on the same
mesh with the manufactured sine right-hand side, the FP64 Jacobi-PCG
time to a 1e-10 relative residual (and the mixed-precision solve when the
library provides it), a plain streaming copy as the achievable-bandwidth
reference, and the CPU oracle on a bounded sample on the host cores.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=2000)
    ap.add_argument("--prewarm-ms", type=float, default=300.0,
                    help="wall time of operator launches run before the warm-up steps, so "
                         "that the timed launches see the sustained clock")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-pcg", action="store_true", help="skip the solver measurements")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--n", type=int, default=32, help="elements per brick edge")
    ap.add_argument("--N", type=int, default=10, help="GLL nodes per direction")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-solve leg")
    ap.add_argument("--nbatch", type=int, default=64, help="problems in the batched leg")
    ap.add_argument("--no-ax-variants", action="store_true",
                    help="skip the FP32 and 16-bit-G AX timings")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the N = 8, 12 solver sweep and the N = 16 AX replay")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-preconditioner leg")
    ap.add_argument("--learned-train", type=int, default=200,
                    help="training meshes (32x16x16, N=10) for the learned leg")
    ap.add_argument("--learned-epochs", type=int, default=8)
    ap.add_argument("--dssum-only", type=int, default=0, metavar="K",
                    help="profiling mode: K dssum passes (FP64, then FP32) on the brick's "
                         "plan and random vectors, then exit")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def src_hash(*names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2011_04981_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def device_record(torch):
    """What the runtime reports about the GPU (to confirm the nominal
    figures the roofline uses)."""
    p = torch.cuda.get_device_properties(0)
    rec = {"name": p.name, "arch": getattr(p, "gcnArchName", None),
           "compute_units": p.multi_processor_count,
           "memory_gib": round(p.total_memory / 2 ** 30, 1)}
    for k in ("L2_cache_size", "clock_rate", "memory_clock_rate", "memory_bus_width"):
        if hasattr(p, k):
            rec[k] = getattr(p, k)
    return rec


def cpu_model():
    """The host CPU's model name, as the kernel reports it."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def traffic_record(kernel_hash):
    """Counter-measured HBM bytes per AX launch, if profiles/ holds a record
    taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "ax_f64_c2_traffic.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_hash") != kernel_hash:
        return None
    return rec.get("hbm_bytes_per_launch")


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "nbx runs on one GPU per process; --gpus must be 1",
                          "n_gpus": a.gpus}), flush=True)
        sys.exit(2)

    import torch
    import synthetic as S
    import paper_2011_04981_amd as nbx

    dev = "cuda"
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    brick = S.Brick(a.n, a.n, a.n, a.N, ((0.05, 2, 2, 2),) * 3, "sine", 0,
                    f"deformed_E{a.n**3}_N{a.N}")
    N, E = brick.N, brick.E
    flops = nbx.ax_flops(N, E)
    abytes = nbx.ax_bytes(N, E)
    out = {}

    if a.dssum_only:
        # the exchange alone, for kernel traces and counters
        gid, bnd = nbx.brick_ids(brick.ex, brick.ey, brick.ez, N)
        gs = nbx.GS(gid, bnd)
        g = torch.Generator(device=dev).manual_seed(0)
        for dt in (torch.float64, torch.float32):
            v = torch.rand(gid.size, dtype=dt, device=dev, generator=g)
            for _ in range(a.dssum_only):
                gs.dssum(v)
            torch.cuda.synchronize()
            log(f"dssum {dt}: {a.dssum_only} passes over {gid.size} local nodes")
        return

    with torch.cuda.stream(stream):
        log(f"set-up: E={E} N={N}")
        D = nbx.deriv_device(N, dev)
        G, bm, _ = nbx.geom_brick(brick.ex, brick.ey, brick.ez, N, brick.deform_array())
        u = torch.as_tensor(S.uniform_field(E, N, seed=0)).to(dev)
        w = torch.empty_like(u)
        stream.synchronize()

        # ---- AX: clock pre-warm, warm-up, then exactly `steps` timed launches.
        # Leaving the idle power state takes ~20 ms of sustained work: per-launch
        # times fall from ~380 to ~315 us over the first ~60 launches, and rise
        # again after an idle second.  A fixed wall time of launches before the
        # warm-up steps puts the timed launches on the sustained clock, whatever
        # the warm-up count.
        pw_launches, pw0 = 0, time.perf_counter()
        while time.perf_counter() - pw0 < a.prewarm_ms * 1e-3:
            for _ in range(8):
                nbx.ax(u, G, D, out=w)
            pw_launches += 8
            stream.synchronize()
        prewarm_ms = (time.perf_counter() - pw0) * 1e3
        for _ in range(a.warmup):
            nbx.ax(u, G, D, out=w)
        stream.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(a.steps)]
        t_all0 = torch.cuda.Event(enable_timing=True)
        t_all1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        h0 = time.perf_counter()
        t_all0.record(stream)
        for k in range(a.steps):
            ev[k][0].record(stream)
            nbx.ax(u, G, D, out=w)
            ev[k][1].record(stream)
        t_all1.record(stream)
        torch.cuda.synchronize()
        h1 = time.perf_counter()
        per = [s.elapsed_time(e) * 1e-3 for s, e in ev]          # seconds per launch
        total = t_all0.elapsed_time(t_all1) * 1e-3
        mean_launch = statistics.fmean(per)
        log(f"AX: mean {mean_launch*1e6:.1f} us  median {statistics.median(per)*1e6:.1f} us  "
            f"min {min(per)*1e6:.1f} us  host {1e6*(h1-h0)/a.steps:.1f} us/step")

        # ---- the same operator on factor pairs (nbx_ax_paired, the layout the
        # solvers keep inside a problem): same bits, three 16-byte factor loads
        # per node instead of six 8-byte ones
        Gp = nbx.pair_factors(G, N)
        for _ in range(20):
            nbx.ax_paired(u, Gp, D, out=w)
        e0 = torch.cuda.Event(enable_timing=True); e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(max(a.steps, 50)):
            nbx.ax_paired(u, Gp, D, out=w)
        e1.record(stream)
        torch.cuda.synchronize()
        paired_launch = e0.elapsed_time(e1) * 1e-3 / max(a.steps, 50)
        del Gp
        log(f"AX on factor pairs: mean {paired_launch*1e6:.1f} us")

        # ---- achievable-bandwidth reference: streaming copy of 1 GiB
        n_copy = (1 << 30) // 8
        src = torch.empty(n_copy, dtype=torch.float64, device=dev).uniform_()
        dst = torch.empty_like(src)
        for _ in range(3):
            nbx.copy_f64(src, dst)
        c0 = torch.cuda.Event(enable_timing=True); c1 = torch.cuda.Event(enable_timing=True)
        c0.record(stream)
        for _ in range(10):
            nbx.copy_f64(src, dst)
        c1.record(stream)
        torch.cuda.synchronize()
        copy_gbs = 2 * 8 * n_copy * 10 / (c0.elapsed_time(c1) * 1e-3) / 1e9
        # two more references: non-temporal copy and a read-only stream
        refs = {}
        sink = torch.zeros(1, dtype=torch.float64, device=dev)
        for mode, name, factor in ((0, "copy_nt_gbs", 2), (1, "read_gbs", 1)):
            for _ in range(3):
                nbx.stream_f64(mode, src, dst, sink)
            c0.record(stream)
            for _ in range(10):
                nbx.stream_f64(mode, src, dst, sink)
            c1.record(stream)
            torch.cuda.synchronize()
            refs[name] = round(factor * 8 * n_copy * 10 / (c0.elapsed_time(c1) * 1e-3) / 1e9, 1)
        log(f"references: non-temporal copy {refs['copy_nt_gbs']:.0f} GB/s, "
            f"read-only {refs['read_gbs']:.0f} GB/s")
        del src, dst
        log(f"copy: {copy_gbs:.0f} GB/s")

        # ---- reduced-precision AX variants (the mixed solve's inner operator)
        variants = {}
        u32 = u.float()
        w32 = torch.empty_like(u32)
        G32 = G.float() if not a.no_ax_variants else None
        runs = {}
        G16f = gsf = G16b = gsb = None
        if not a.no_ax_variants:
            runs["fp32"] = (lambda: nbx.ax(u32, G32, D, out=w32), 32)
            G16f, gsf = nbx.g16_pack(G, N, nbx.F16)
            G16b, gsb = nbx.g16_pack(G, N, nbx.BF16)
            runs["g_fp16"] = (lambda: nbx.ax_g16(u32, G16f, gsf, D, nbx.F16, out=w32), 20)
            runs["g_bf16"] = (lambda: nbx.ax_g16(u32, G16b, gsb, D, nbx.BF16, out=w32), 20)
            # the same operators on matrix cores (FP32 products and accumulation)
            runs["mfma_fp32"] = (lambda: nbx.ax_mfma(u32, G32, D, out=w32), 32)
            runs["mfma_g_fp16"] = (lambda: nbx.ax_mfma(u32, G16f, D, gprec=nbx.F16, gscale=gsf,
                                                       out=w32), 20)
        for name, (fn, bpn) in runs.items():
            for _ in range(50):
                fn()
            e0 = torch.cuda.Event(enable_timing=True); e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(200):
                fn()
            e1.record(stream)
            torch.cuda.synchronize()
            t = e0.elapsed_time(e1) * 1e-3 / 200
            gbs = bpn * E * N ** 3 / t / 1e9
            variants[name] = {"mean_launch_us": round(t * 1e6, 2), "bytes_per_node": bpn,
                              "achieved_gbs": round(gbs, 1),
                              "frac": round(gbs / PEAK_HBM_GBS, 4),
                              "gflops": round(flops / t / 1e9, 1)}
            log(f"AX {name}: {t*1e6:.1f} us, {gbs:.0f} GB/s")
        del u32, w32, G32, G16f, gsf, G16b, gsb

        # ---- host -> device transfer of the operator's inputs (G and u) from
        # pinned host memory, against the AX time: how many applications one
        # transfer must serve to be negligible (the library itself builds G
        # on the device, so no transfer is on any timed path)
        transfer = None
        if not a.no_ax_variants:
            hG = torch.empty(G.shape, dtype=G.dtype, pin_memory=True)
            hu = torch.empty(u.shape, dtype=u.dtype, pin_memory=True)
            dG = torch.empty_like(G)
            du = torch.empty_like(u)
            dG.copy_(hG, non_blocking=True)
            du.copy_(hu, non_blocking=True)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True); e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(3):
                dG.copy_(hG, non_blocking=True)
                du.copy_(hu, non_blocking=True)
            e1.record(stream)
            torch.cuda.synchronize()
            t_h2d = e0.elapsed_time(e1) * 1e-3 / 3
            nbytes = (G.numel() + u.numel()) * 8
            transfer = {"bytes": nbytes, "seconds": round(t_h2d, 5),
                        "gbs": round(nbytes / t_h2d / 1e9, 1),
                        "ax_applications_per_transfer": round(t_h2d / mean_launch, 1)}
            log(f"H2D of G and u: {t_h2d*1e3:.1f} ms = {transfer['gbs']:.0f} GB/s "
                f"= {transfer['ax_applications_per_transfer']:.0f} AX applications")
            del hG, hu, dG, du

    ax_hash = src_hash("ax_kernel.hpp", "ax_planes.hip", "ax.hip")
    achieved = abytes / mean_launch / 1e9
    tb = traffic_record(ax_hash) if (N, E) == (10, 32768) else None
    value = flops * a.steps / total / 1e9
    out.update({
        "metric": "AX GFLOP/s + % HBM roofline at N=10; PCG time-to-1e-10 vs plain FP64 Jacobi",
        "value": round(value, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(total / a.steps * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"AX on a {a.n}x{a.n}x{a.n} deformed brick (E={E}), N={N}, "
                               "full 6-factor G in FP64 as [E][6][N^3], u~U[-1,1] seed 0",
                   "E": E, "N": N, "flops_per_step": flops, "hbm_bytes_per_step": abytes},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                     # counter-measured HBM bytes per launch / mean launch time
                     "traffic": (round(tb / mean_launch / 1e9, 1) if tb else None),
                     "traffic_bytes_per_launch": tb,
                     "algorithmic_bytes_per_launch": abytes,
                     "kernel": f"ax_kernel<double,{N},{nbx.get_tile(nbx.F64, N)},false,"
                               "double,true>",
                     "entry_point": "nbx_ax (G as [E][6][N^3], one plane per factor)",
                     "kernel_source_hash": ax_hash,
                     "mean_launch_us": round(mean_launch * 1e6, 2),
                     "median_launch_us": round(statistics.median(per) * 1e6, 2),
                     "min_launch_us": round(min(per) * 1e6, 2),
                     "max_launch_us": round(max(per) * 1e6, 2),
                     # each timed launch in launch order (HIP events on the
                     # launch stream), to show where slow launches sit
                     "launch_us_in_order": ([round(x * 1e6, 1) for x in per]
                                            if len(per) <= 100 else None),
                     "prewarm_ms": round(prewarm_ms, 1),
                     "prewarm_launches": pw_launches,
                     "paired_layout": {
                         "entry_point": "nbx_ax_paired (G as [E][3][N^3][2] factor pairs)",
                         "mean_launch_us": round(paired_launch * 1e6, 2),
                         "achieved": round(abytes / paired_launch / 1e9, 1),
                         "frac": round(abytes / paired_launch / 1e9 / PEAK_HBM_GBS, 4)},
                     "copy_gbs": round(copy_gbs, 1),
                     "frac_of_copy": round(achieved / copy_gbs, 4),
                     **refs,
                     "frac_of_read": round(achieved / refs["read_gbs"], 4)},
        "ax_reduced_precision": variants,
        "host_to_device": transfer,
        "device": device_record(torch),
    })
    del u, w, G, bm
    torch.cuda.empty_cache()

    # ---- solver: FP64 Jacobi-PCG to 1e-10 (and mixed precision if present)
    if not a.no_pcg:
        with torch.cuda.stream(stream):
            log("solver set-up")
            st = nbx.setup_brick(brick.ex, brick.ey, brick.ez, N, brick.deform_array())
            stream.synchronize()
            pcg = {}
            x, r = st.problem.pcg(st.b, rtol=1e-10, max_iter=5000, check_every=20)
            times = []
            for _ in range(3):
                h0 = time.perf_counter()
                x, r = st.problem.pcg(st.b, rtol=1e-10, max_iter=5000, check_every=20)
                times.append(time.perf_counter() - h0)
            pcg["fp64"] = {"iters": r.iters, "seconds": round(min(times), 5),
                           "loop_seconds": round(r.seconds, 5), "relres": r.relres,
                           "true_relres": r.true_relres, "status": r.status}
            log(f"FP64 PCG: {r.iters} it, {min(times):.4f} s, true relres {r.true_relres:.2e}")
            x64 = x.clone()
            _, r100 = st.problem.pcg(st.b, max_iter=100, fixed_iters=1, check_every=20)
            pcg["fp64_100_iterations_seconds"] = round(r100.seconds, 5)
            pcg["fused_stage_tile"] = {"f64": nbx.get_pcg_tile(nbx.F64, N),
                                       "f32": nbx.get_pcg_tile(nbx.F32, N)}
            pcg["ms_per_iteration"] = round(r100.seconds / 100 * 1e3, 4)
            variants = {"mixed_fp32": dict(prec=nbx.F32, mixed_mode=0, inner_rtol=0.1),
                        "mixed_fp32_restarted": dict(prec=nbx.F32, mixed_mode=1,
                                                     inner_rtol=1e-5),
                        "mixed_f16_storage": dict(prec=nbx.F16, mixed_mode=0, inner_rtol=0.1),
                        "mixed_fp32_mfma": dict(prec=nbx.F32, mixed_mode=0, inner_rtol=0.1,
                                                inner_mfma=1),
                        "mixed_f16_storage_mfma": dict(prec=nbx.F16, mixed_mode=0,
                                                       inner_rtol=0.1, inner_mfma=1),
                        "mixed_bf16_storage": dict(prec=nbx.BF16, mixed_mode=0,
                                                   inner_rtol=0.1)}
            for name, kw in variants.items():
                try:
                    times = []
                    for _ in range(3):
                        h0 = time.perf_counter()
                        xm, rm = st.problem.pcg(st.b, rtol=1e-10, max_iter=10000,
                                                check_every=20, **kw)
                        times.append(time.perf_counter() - h0)
                    err = float((xm - x64).abs().max() / x64.abs().max())
                    pcg[name] = {"iters": rm.iters, "outer": rm.outer_iters,
                                 "seconds": round(min(times), 5),
                                 "true_relres": rm.true_relres, "fell_back": rm.fell_back,
                                 "err_vs_fp64": err, "err_reference": "this run's FP64 GPU solve", "status": rm.status,
                                 "speedup_vs_fp64": round(pcg["fp64"]["seconds"] / min(times),
                                                          3),
                                 "inner": {nbx.F32: "fp32", nbx.F16: "G in fp16, fp32 vectors",
                                           nbx.BF16: "G in bf16, fp32 vectors"}[kw["prec"]]
                                          + (", operator on matrix cores"
                                             if kw.get("inner_mfma") else ""),
                                 "mixed_mode": kw["mixed_mode"],
                                 "inner_rtol": kw["inner_rtol"]}
                    log(f"{name}: {rm.iters} it / {rm.outer_iters} outer, {min(times):.4f} s")
                except nbx.NbxError as e:
                    pcg[name] = {"unavailable": str(e)}
            out["pcg"] = pcg
            del st, x, x64
            torch.cuda.empty_cache()

    # ---- C1: the 4x4x4 affine brick at N = 10 (4 MB working set, cache
    # resident): AX and 100 FP64 PCG iterations
    if not a.no_pcg and a.N == 10:
        with torch.cuda.stream(stream):
            c1 = S.c1_brick()
            st1 = nbx.setup_brick(c1.ex, c1.ey, c1.ez, c1.N)
            u1 = torch.as_tensor(S.uniform_field(c1.E, c1.N, seed=0)).to(dev)
            w1 = torch.empty_like(u1)
            for _ in range(50):
                nbx.ax(u1, st1.G, st1.D, out=w1)
            per1 = []
            for _ in range(100):
                e0 = torch.cuda.Event(enable_timing=True); e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                nbx.ax(u1, st1.G, st1.D, out=w1)
                e1.record(stream)
                per1.append((e0, e1))
            torch.cuda.synchronize()
            t1 = statistics.median(s_.elapsed_time(e_) * 1e-3 for s_, e_ in per1)
            # back to back: 200 launches between two events (per-launch
            # events above also time the host's submission gaps)
            e0 = torch.cuda.Event(enable_timing=True); e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(200):
                nbx.ax(u1, st1.G, st1.D, out=w1)
            e1.record(stream)
            torch.cuda.synchronize()
            t1b = e0.elapsed_time(e1) * 1e-3 / 200
            # cold: a 512 MB copy before each launch evicts the 4 MB working
            # set from L2 and MALL
            fa = torch.empty(64 << 20, dtype=torch.float64, device=dev)
            fb = torch.empty_like(fa)
            per1c = []
            for _ in range(20):
                nbx.copy_f64(fa, fb)
                e0 = torch.cuda.Event(enable_timing=True); e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                nbx.ax(u1, st1.G, st1.D, out=w1)
                e1.record(stream)
                per1c.append((e0, e1))
            torch.cuda.synchronize()
            t1c = statistics.median(s_.elapsed_time(e_) * 1e-3 for s_, e_ in per1c)
            del fa, fb
            st1.problem.pcg(st1.b, max_iter=100, fixed_iters=1, check_every=20)
            _, r1 = st1.problem.pcg(st1.b, max_iter=100, fixed_iters=1, check_every=20)
            out["c1"] = {"E": c1.E, "N": 10, "ax_median_us": round(t1 * 1e6, 2),
                         "ax_gflops": round(nbx.ax_flops(10, c1.E) / t1 / 1e9, 1),
                         "ax_caches": "warm (repeated launches on a 4 MB working set)",
                         "ax_back_to_back_us": round(t1b * 1e6, 2),
                         "ax_back_to_back_gflops": round(nbx.ax_flops(10, c1.E) / t1b / 1e9, 1),
                         "ax_cold_median_us": round(t1c * 1e6, 2),
                         "ax_cold_gflops": round(nbx.ax_flops(10, c1.E) / t1c / 1e9, 1),
                         "pcg_100_iterations_seconds": round(r1.seconds, 5)}
            log(f"C1: AX {t1*1e6:.1f} us warm, {t1b*1e6:.1f} us back to back, "
                f"{t1c*1e6:.1f} us cold, "
                f"100 PCG iterations {r1.seconds*1e3:.2f} ms")
            del st1, u1, w1

    # ---- the same mesh at N = 8 and 12: FP64 PCG against the refinement
    # variants (N = 10 is the block above); and the paper's own element
    # size, N = 16, for the plain operator at E = 800 and E = 8000
    # (--no-pcg keeps the operator replay and skips the solves)
    if not a.no_sweep and a.N == 10:
        sweep = {}
        with torch.cuda.stream(stream):
            for Ns in ((8, 12) if not a.no_pcg else ()):
                log(f"sweep: N={Ns}")
                st = nbx.setup_brick(brick.ex, brick.ey, brick.ez, Ns, brick.deform_array())
                stream.synchronize()
                row = {}
                x64 = None
                for name, kw in (("fp64", dict(prec=nbx.F64)),
                                 ("mixed_fp32", dict(prec=nbx.F32, mixed_mode=0,
                                                     inner_rtol=0.1)),
                                 ("mixed_f16_storage", dict(prec=nbx.F16, mixed_mode=0,
                                                            inner_rtol=0.1))):
                    st.problem.pcg(st.b, rtol=1e-10, max_iter=20000, check_every=20, **kw)
                    times = []
                    for _ in range(2):
                        h0 = time.perf_counter()
                        xs, rs = st.problem.pcg(st.b, rtol=1e-10, max_iter=20000,
                                                check_every=20, **kw)
                        times.append(time.perf_counter() - h0)
                    rec = {"iters": rs.iters, "outer": rs.outer_iters,
                           "seconds": round(min(times), 5), "true_relres": rs.true_relres,
                           "fell_back": rs.fell_back, "status": rs.status}
                    if x64 is None:
                        x64 = xs.clone()
                    else:
                        rec["err_vs_fp64"] = float((xs - x64).abs().max() / x64.abs().max())
                        rec["speedup_vs_fp64"] = round(row["fp64"]["seconds"] / min(times), 3)
                    row[name] = rec
                    log(f"  N={Ns} {name}: {rs.iters} it, {min(times):.3f} s")
                sweep[f"N{Ns}"] = {"E": E, "local_nodes": E * Ns ** 3, **row}
                del st, x64, xs
                torch.cuda.empty_cache()
            if not a.no_pcg:
                # the paper's element size in a solve: FP64 Jacobi-PCG on the
                # C2 deformation over a 20^3 brick at N = 16 (E = 8000, the
                # replay's larger size; the fused stage on the matrix cores)
                b16 = S.scaled_c2_brick(20, 16)
                log(f"sweep: N=16, E={b16.E}")
                st = nbx.setup_brick(b16.ex, b16.ey, b16.ez, 16, b16.deform_array())
                stream.synchronize()
                st.problem.pcg(st.b, rtol=1e-10, max_iter=20000, check_every=20)
                times = []
                for _ in range(2):
                    h0 = time.perf_counter()
                    _, rs = st.problem.pcg(st.b, rtol=1e-10, max_iter=20000, check_every=20)
                    times.append(time.perf_counter() - h0)
                sweep["N16"] = {"E": b16.E, "local_nodes": b16.E * 16 ** 3,
                                "fp64": {"iters": rs.iters, "seconds": round(min(times), 5),
                                         "ms_per_iter": round(min(times) / rs.iters * 1e3, 4),
                                         "true_relres": rs.true_relres, "status": rs.status}}
                log(f"  N=16 fp64: {rs.iters} it, {min(times):.3f} s")
                del st
                torch.cuda.empty_cache()
            replay = {}
            for Er in (800, 8000):
                Nr = 16
                ur = torch.as_tensor(S.uniform_field(Er, Nr, seed=0)).to(dev)
                Gr = torch.as_tensor(S.random_factors(Er, Nr, seed=1)).to(dev)
                Dr = nbx.deriv_device(Nr, dev)
                wr = torch.empty_like(ur)
                # nbx_ax (FP64 N = 16 runs on the matrix cores), then the
                # vector-unit kernel (an explicit tile) on the same inputs
                ts = {}
                for kind, kw in (("mfma", {}), ("vector", {"epb": 1})):
                    for _ in range(20):
                        nbx.ax(ur, Gr, Dr, out=wr, **kw)
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                    for _ in range(100):
                        nbx.ax(ur, Gr, Dr, out=wr, **kw)
                    e1.record(stream)
                    torch.cuda.synchronize()
                    ts[kind] = e0.elapsed_time(e1) * 1e-3 / 100
                t = ts["mfma"]
                replay[f"E{Er}"] = {
                    "N": Nr, "kernel": "ax16_mfma_kernel (matrix cores)",
                    "mean_launch_us": round(t * 1e6, 2),
                    "gflops": round(nbx.ax_flops(Nr, Er) / t / 1e9, 1),
                    "gbs_algorithmic": round(nbx.ax_bytes(Nr, Er) / t / 1e9, 1),
                    "frac_hbm_peak": round(nbx.ax_bytes(Nr, Er) / t / 1e9 / PEAK_HBM_GBS, 4),
                    "vector_unit_kernel_us": round(ts["vector"] * 1e6, 2),
                    "speedup_vs_vector_unit": round(ts["vector"] / t, 3),
                    "working_set_mb": round(nbx.ax_bytes(Nr, Er) / 1e6, 1)}
                if Er == 800:
                    # the paper's own measurement (FP64 AX, 16 points per
                    # direction, E = 800; Table II and Section IV), other
                    # hardware: context for this line, not its target
                    replay["E800"]["paper_context_gflops"] = {
                        "V100": 407.62, "U280_4_kernels": 289.02, "Xeon_8260M_24_cores": 65.74}
                log(f"  AX N=16 E={Er}: {t*1e6:.1f} us (vector-unit kernel "
                    f"{ts['vector']*1e6:.1f} us)")
                del ur, Gr, wr
            out["sweep"] = {"solvers": sweep, "ax_n16_paper_sizes": replay}
            torch.cuda.empty_cache()

    # ---- batched solves: independent problems of uneven E and N together
    if not a.no_batched:
        with torch.cuda.stream(stream):
            log(f"batched set-up: {a.nbatch} problems")
            specs = S.c4_problems(a.nbatch)
            sets = [nbx.setup_brick(b.ex, b.ey, b.ez, b.N, b.deform_array(),
                                    f=torch.as_tensor(S.rhs_values(b)).to(dev)) for b in specs]
            stream.synchronize()
            probs = [s_.problem for s_ in sets]
            bs = [s_.b for s_ in sets]
            nbx.pcg_batched(probs, bs, rtol=1e-10, max_iter=5000, check_every=20)
            h0 = time.perf_counter()
            xs, res, lat = nbx.pcg_batched(probs, bs, rtol=1e-10, max_iter=5000, check_every=20)
            wall = time.perf_counter() - h0
            # the same problems one after another with the standalone solver
            h1 = time.perf_counter()
            seq_iters = []
            for s_ in sets:
                _, r1 = s_.problem.pcg(s_.b, rtol=1e-10, max_iter=5000, check_every=20)
                seq_iters.append(r1.iters)
            seq = time.perf_counter() - h1
            flops = sum(r.iters * nbx.ax_flops(b.N, b.E) for r, b in zip(res, specs))
            lat_sorted = sorted(lat)
            pct = lambda q: lat_sorted[min(len(lat_sorted) - 1, int(q * len(lat_sorted)))]
            out["batched"] = {
                "problems": len(specs), "nodes": int(sum(b.n_local for b in specs)),
                "converged": int(sum(r.flag == 1 for r in res)),
                "same_iterations_as_standalone": bool(all(r.iters == i for r, i
                                                          in zip(res, seq_iters))),
                "wall_seconds": round(wall, 4), "sequential_seconds": round(seq, 4),
                "speedup_vs_sequential": round(seq / wall, 3),
                "ax_gflops_aggregate": round(flops / wall / 1e9, 1),
                "latency_p50_s": round(pct(0.50), 5), "latency_p99_s": round(pct(0.99), 5),
                "latency_max_s": round(lat_sorted[-1], 5),
                "iterations_min_max": [min(r.iters for r in res), max(r.iters for r in res)],
                "fused_stage_tiles": {str(N): nbx.get_pcg_tile(nbx.F64, N)
                                      for N in (6, 8, 10, 12)}}
            log(f"batched: {wall:.3f} s vs sequential {seq:.3f} s, "
                f"p50 {pct(0.5):.4f} s p99 {pct(0.99):.4f} s")
            # the same batch with FP16-stored G in the inner iterations
            # (reliable updates; per-solve latency from the host)
            kw16 = dict(rtol=1e-10, max_iter=10000, check_every=20, prec=nbx.F16,
                        inner_rtol=0.1)
            try:
                nbx.pcg_batched(probs, bs, **kw16)
                h0 = time.perf_counter()
                xm, resm, latm = nbx.pcg_batched(probs, bs, **kw16)
                wallm = time.perf_counter() - h0
                errm = max(float((a_ - b_).abs().max() / b_.abs().max())
                           for a_, b_ in zip(xm, xs))
                latm_sorted = sorted(latm)
                pctm = lambda q: latm_sorted[min(len(latm_sorted) - 1,
                                                 int(q * len(latm_sorted)))]
                out["batched"]["mixed_f16_storage"] = {
                    "wall_seconds": round(wallm, 4),
                    "speedup_vs_fp64_batch": round(wall / wallm, 3),
                    "converged": int(sum(r.flag == 1 for r in resm)),
                    "max_true_relres": max(r.true_relres for r in resm),
                    "fell_back": int(sum(r.fell_back for r in resm)),
                    "max_err_vs_fp64_batch": errm,
                    "latency_p50_s": round(pctm(0.50), 5),
                    "latency_p99_s": round(pctm(0.99), 5)}
                log(f"batched FP16-G mixed: {wallm:.3f} s, p50 {pctm(0.5):.4f} s, "
                    f"p99 {pctm(0.99):.4f} s, max true relres "
                    f"{max(r.true_relres for r in resm):.2e}")
                del xm
            except nbx.NbxError as e:
                out["batched"]["mixed_f16_storage"] = {"unavailable": str(e)}
            del sets, probs, bs, xs
            torch.cuda.empty_cache()

    # ---- learned element-local preconditioner: train on FP64-CG samples,
    # pick the damping on a validation brick, compare with Jacobi-PCG on an
    # unseen 32^3 brick
    if not a.no_learned and a.N == 10:
        from paper_2011_04981_amd import learned as LL
        with torch.cuda.stream(stream):
            log(f"learned preconditioner: training on {a.learned_train} meshes")
            ev = [S.Brick(a.n, a.n, a.n, 10, S.deformation_family(10000), "random", 10000,
                          f"eval10000_E{a.n**3}")]
            out["learned"] = LL.run_c5(n_train=a.learned_train, epochs=a.learned_epochs,
                                       eval_meshes=ev, log=log)
            torch.cuda.empty_cache()

    # ---- CPU oracle baseline (host cores, bounded sample)
    if not a.no_cpu:
        import oracle as O
        ez = max(1, 4096 // (a.n * a.n))
        sb = S.Brick(a.n, a.n, ez, N, brick.deform, "sine", 0)
        xi, wq = O.gll(N)
        Do = O.deriv(N, xi)
        Go, _, _ = O.geom(N, Do, wq, *O.brick_coords(sb, xi))
        uo = S.uniform_field(sb.E, N, seed=0)
        O.ax(uo, Go, Do)
        reps, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < a.cpu_seconds and reps < 100000:
            O.ax(uo, Go, Do)
            reps += 1
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {
            "value": round(nbx.ax_flops(N, sb.E) * reps / dt / 1e9, 3), "unit": "GFLOP/s",
            "cores": O.num_threads(), "kind": "oracle", "cpu_model": cpu_model(),
            "affinity_cores": len(os.sched_getaffinity(0)),
            "sample": f"oracle AX on {sb.E} elements ({a.n}x{a.n}x{ez} slab of the same "
                      f"deformed mapping, N={N}), {reps} applications in {dt:.1f} s"}
        log(f"cpu oracle: {out['cpu_baseline']['value']} GFLOP/s on {O.num_threads()} threads")
        # the small affine brick C1 (4x4x4, N = 10) on one core and on all, 100
        # oracle PCG iterations on C1, and the oracle's PCG iteration on the
        # benchmark brick
        c1 = S.c1_brick()
        P1 = O.setup(c1)
        u1 = S.uniform_field(c1.E, c1.N, seed=0)
        extra = {}
        all_threads = O.num_threads()
        for label, nt in (("1core", 1), ("allcores", all_threads)):
            O.set_num_threads(nt)
            O.ax(u1, P1.G, P1.D)
            reps, t0 = 0, time.perf_counter()
            while time.perf_counter() - t0 < 1.0:
                O.ax(u1, P1.G, P1.D)
                reps += 1
            dt = time.perf_counter() - t0
            extra[f"c1_ax_gflops_{label}"] = round(nbx.ax_flops(10, c1.E) * reps / dt / 1e9, 3)
        O.set_num_threads(all_threads)
        h0 = time.perf_counter()
        O.pcg(P1, max_iter=100, rtol=0.0)
        extra["c1_pcg_100_iterations_seconds"] = round(time.perf_counter() - h0, 4)
        if (a.n, a.N) == (32, 10):
            # 10 iterations (a bounded sample), reported per iteration
            P2 = O.setup(brick)
            h0 = time.perf_counter()
            O.pcg(P2, max_iter=10, rtol=0.0)
            per_it = (time.perf_counter() - h0) / 10
            extra["c2_pcg_seconds_per_iteration"] = round(per_it, 4)
            fp64 = out.get("pcg", {}).get("fp64")
            if fp64:
                # projection, not a measurement: the oracle's PCG takes the GPU's
                # iteration count to within one on every mesh both solve
                extra["c2_time_to_1e-10_projected_seconds"] = round(per_it * fp64["iters"], 1)
                extra["c2_time_to_1e-10_projection"] = (
                    f"{per_it:.4f} s per oracle iteration (10 timed) x {fp64['iters']} "
                    "iterations of the GPU's FP64 solve")
            del P2
        out["cpu_baseline"]["extra"] = extra
        log(f"cpu oracle extra: {extra}")

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
