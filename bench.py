#!/usr/bin/env python3
"""Throughput benchmark of the curvilinear AFWENO Navier-Stokes RK3 step on one MI355X.

A step is one full TVD-RK3 step (three fused RHS + stage evaluations and the halo
exchanges after each stage) over the whole grid.  The metric is grid-point RK3 stage
updates per second: interior points x 3 stages x steps / wall time of the timed steps.

Default workload: 256^3 periodic Taylor-Green vortex, Mach 0.1, Re 1600, on the 2 pi cube
with a sinusoidal grid perturbation of amplitude 0.05 and seeded velocity noise, FP64.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
                       [--workload tgv256|vortex32|ogrid24|channel]
                       [--precision fp64|mixed] [--form single|perblock|batched] [--no-cpu]
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import re
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# algorithmic HBM bytes per interior point of each kernel (compulsory reads and writes)
# FP64 path: Q 40 B, a metric component or J 8 B, a viscous-flux component 8 B
# compulsory HBM bytes per interior point of each kernel, by the role of a sweep in the
# direction order (first: no partial sum in; last: the RK combination)
ALG_BYTES_FP64 = {
    "visc_prepass": 40 + 80 + 96,          # Q, 9 metrics + J, 12 flux planes
    "first": 40 + 24 + 32 + 40,            # Q, 3 metrics, 4 flux planes, partial sum out
    "middle": 40 + 24 + 32 + 40 + 40,      # + partial sum in
    "last_rk": 40 + 24 + 32 + 40 + 8 + 40 + 40,  # Q, metrics, fluxes, partial in, J, Qn, Qout
}
ALG_BYTES_MIXED = {
    "visc_prepass": 40 + 40 + 48,          # Q, the FP32 copy of the metrics, FP32 flux planes
    "first": 40 + 24 + 16 + 20,
    "middle": 40 + 24 + 16 + 20 + 20,
    "last_rk": 40 + 24 + 16 + 20 + 8 + 40 + 40,
}
DIR_NAMES = ("xi", "eta", "zeta")


def kernel_bytes(table, order):
    """Algorithmic bytes per point keyed by the library's profiler names."""
    out = {"visc_prepass": table["visc_prepass"]}
    out[f"sweep_{DIR_NAMES[order[0]]}"] = table["first"]
    out[f"sweep_{DIR_NAMES[order[1]]}"] = table["middle"]
    out[f"sweep_{DIR_NAMES[order[2]]}_rk"] = table["last_rk"]
    return out


HBM_PEAK_GBS = 8000.0


def _code_only(text: str) -> str:
    """Source text without comments and whitespace runs (a comment edit changes no kernel)."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def source_sha() -> str:
    """Hash of the kernel and library sources (code only), to tie measured counters to them."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2006_07964_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), encoding="utf-8") as fh:
            h.update(name.encode())
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def load_traffic(kernel: str, workload: str, precision: str):
    """Measured HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled by a copy
    kernel's reading) if they were taken on the current kernel sources, else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        data = json.load(open(path))
    except ValueError:
        return None
    ent = data.get(f"{workload}/{precision}/{kernel}")
    if not ent or ent.get("source_sha") != source_sha():
        return None
    return ent.get("bytes_per_launch")


WORKLOADS = {
    "tgv256": "taylor_green_256^3_wavy_2pi_mach0.1_re1600",
    "vortex32": "isentropic_vortex_32^3_wavy_unit_mach0.5_re1000",
    "ogrid24": "o_grid_24_uneven_blocks_mach0.2_vortices_wall_farfield",
    "channel": "channel_512x512x384_tanh2.5_bump0.02_mach0.3",
}


def build_workload(name: str):
    from paper_2006_07964_amd import workloads as W
    if name == "tgv256":
        return W.taylor_green_wavy(256), WORKLOADS[name]
    if name == "vortex32":
        return W.vortex_wavy(32), WORKLOADS[name]
    if name == "ogrid24":
        wl = W.o_grid_vortices()
        return wl, WORKLOADS[name] + f"_{wl.points}pts"
    if name == "channel":
        return W.channel(), WORKLOADS[name]
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(wl, workload_name, scheme=0):
    """The oracle, as it stands, timed on the host: one full RK3 step (three stages) of the
    same workload with the same inviscid scheme."""
    import oracle as O
    b = wl.blocks[0]
    c = O.cfg_from_workload(wl, scheme=scheme)
    met = O.metrics(c, b.xyz)
    dt = O.dt_cfl(c, met, b.q, wl.cfl)
    t0 = time.perf_counter()
    O.rk_step(c, met, dt, b.q)
    el = time.perf_counter() - t0
    return {"value": 3 * b.points / el, "unit": "updates/s", "cores": O.threads(),
            "kind": "oracle",
            "sample": f"one RK3 step (3 stages: RHS + update + halo wrap) of the full {workload_name} grid, "
                      f"{el:.2f} s on {O.threads()} OpenMP threads"}


def cpu_baseline_one_thread(workload: str, scheme=0):
    """The oracle on one thread (the paper quotes its speed-up over one CPU core): one full
    RK3 step of a smaller instance of the same workload (same scheme, same arithmetic per
    point; the full-size step would take minutes on one core), as updates/s."""
    import oracle as O
    from paper_2006_07964_amd import workloads as W
    small = {"tgv256": lambda: W.taylor_green_wavy(128), "vortex32": lambda: W.vortex_wavy(32),
             "channel": lambda: W.channel(128, 128, 96)}.get(workload)
    if small is None:
        return None
    wl = small()
    b = wl.blocks[0]
    c = O.cfg_from_workload(wl, scheme=scheme)
    met = O.metrics(c, b.xyz)
    dt = O.dt_cfl(c, met, b.q, wl.cfl)
    before = O.set_threads(1)
    try:
        t0 = time.perf_counter()
        O.rk_step(c, met, dt, b.q)
        el = time.perf_counter() - t0
    finally:
        O.set_threads(before)
    return {"value": 3 * b.points / el, "unit": "updates/s", "cores": 1, "kind": "oracle",
            "sample": f"one RK3 step of the {b.ni}x{b.nj}x{b.nk} instance of the same workload, "
                      f"{el:.2f} s on 1 thread"}


def copy_bandwidth(torch):
    """Achievable HBM bandwidth of a plain device copy (GB/s, read + write bytes)."""
    n = 1 << 27  # 1 GiB of float64
    a = torch.empty(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    reps = 10
    for _ in range(reps):
        b.copy_(a)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    del a, b
    return 2 * n * 8 / (ms * 1e-3) / 1e9


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="tgv256")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--form", default=None, choices=["single", "perblock", "batched"],
                    help="single-block calls, per-block launches, or the batched graph form")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--scheme", default="modified", choices=["modified", "original"],
                    help="inviscid scheme: modified AFWENO (characteristic space at the nodes) or the "
                         "original one (at the half points)")
    ap.add_argument("--tiles", default=None,
                    help="sweep tile shapes xi,eta,zeta of the single / per-block forms (library default if unset)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-block path runs all blocks on one device)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2006_07964_amd import binding as B

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    torch.cuda.set_device(0)
    B.lib()
    wl, wname = build_workload(args.workload)
    prec = B.CFD_FP64 if args.precision == "fp64" else B.CFD_MIXED
    stream = torch.cuda.current_stream()
    nb = len(wl.blocks)
    form = args.form or ("single" if nb == 1 else "perblock")
    if form == "single" and nb != 1:
        raise SystemExit("--form single needs a single-block workload")
    scheme = B.CFD_AFWENO_ORIGINAL if args.scheme == "original" else B.CFD_AFWENO_MODIFIED
    descs, hs, qs, qas, qbs = [], [], [], [], []
    for bi, blk in enumerate(wl.blocks):
        # rows padded to 16 doubles and offset so that interior rows start 128-byte lines
        desc = B.desc_from_workload(wl, bi, prec, ld_i=B.aligned_pitch(blk.ni), scheme=scheme)
        h = B.cfd_block_create(desc, stream)
        if args.tiles:
            B.cfd_block_set_tiles(h, [int(v) for v in args.tiles.split(",")])
        xyz = torch.from_numpy(blk.xyz).cuda()
        B.cfd_metrics(h, xyz, blk.ni + 12, blk.nj + 12)
        del xyz
        descs.append(desc)
        hs.append(h)
        qs.append(B.upload_state(desc, blk.q))
        qas.append(B.upload_state(desc, blk.q))
        qbs.append(B.upload_state(desc, blk.q))
    x = B.cfd_exchange_create(hs, wl.interfaces)
    B.cfd_halo_exchange(x, B.CFD_FIELDS_Q, qs)
    dt = B.cfd_dt_cfl(hs, qs, wl.cfl)
    dt_dev = torch.tensor([dt], dtype=torch.float64, device="cuda")
    points = wl.points
    bt = None
    if form == "batched":
        bt = B.cfd_batch_create(hs, x, stream)
    h = hs[0]
    q, qa, qb = qs[0], qas[0], qbs[0]
    blk = wl.blocks[0]

    def stage(st, cur, out):
        for hb, c in zip(hs, cur):
            B.cfd_viscous_fluxes(hb, c)
        B.cfd_halo_exchange(x, B.CFD_FIELDS_VISC, None)
        for hb, qn, c, o in zip(hs, qs, cur, out):
            B.cfd_rk_sweeps(hb, st, dt, qn, c, o)
        B.cfd_halo_exchange(x, B.CFD_FIELDS_Q, out)

    def step():
        if form == "batched":
            B.cfd_batch_step(bt, dt_dev, qs, qas, qbs)
        elif form == "perblock":
            stage(0, qs, qas)
            stage(1, qas, qbs)
            stage(2, qbs, qs)
        else:
            B.cfd_rk_stage(h, 0, dt, q, q, qa)
            B.cfd_halo_exchange(x, B.CFD_FIELDS_Q, [qa])
            B.cfd_rk_stage(h, 1, dt, q, qa, qb)
            B.cfd_halo_exchange(x, B.CFD_FIELDS_Q, [qb])
            B.cfd_rk_stage(h, 2, dt, q, qb, q)
            B.cfd_halo_exchange(x, B.CFD_FIELDS_Q, [q])

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    profiled = form != "batched"  # a captured graph is timed as a whole
    for hb in hs:
        B.cfd_profile_reset(hb)
        B.cfd_profile_enable(hb, profiled)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for n in range(args.steps):
        step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = {}
    for hb in hs:
        B.cfd_profile_enable(hb, False)
        for name, (launches, ms) in B.cfd_profile_read(hb).items():
            l0, m0 = prof.get(name, (0, 0.0))
            prof[name] = (l0 + launches, m0 + ms)
    for hb, qb_ in zip(hs, qs):
        if not B.cfd_check_finite(hb, qb_):
            raise SystemExit("non-finite state after the timed steps")
    updates = points * 3 * args.steps
    value = updates / el

    alg = kernel_bytes(ALG_BYTES_FP64 if prec == B.CFD_FP64 else ALG_BYTES_MIXED, B.cfd_sweep_order())
    stage_bytes = sum(alg.values()) * points
    kernels = {}
    for name, (launches, ms) in prof.items():
        avg_ms = ms / max(launches, 1)
        ent = {"launches": launches, "avg_ms": round(avg_ms, 4), "share": 0.0}
        if name in alg:
            # each block launches every kernel equally often
            total_bytes = alg[name] * points * launches / nb
            ent["alg_bytes_per_launch"] = int(total_bytes / launches)
            ent["alg_GBps"] = round(total_bytes / (ms * 1e-3) / 1e9, 1)
        kernels[name] = ent
    total_ms = sum(v[1] for v in prof.values())
    for name, ent in kernels.items():
        ent["share"] = round(prof[name][1] / total_ms, 3)
    if kernels:
        dom = max((n for n in kernels if n in alg), key=lambda n: prof[n][1])
        dk = kernels[dom]
        achieved = dk["alg_GBps"]
        roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": load_traffic(dom, args.workload, args.precision), "kernel": dom,
                    "alg_bytes_per_point": alg[dom], "avg_launch_ms": dk["avg_ms"]}
    else:  # a captured graph: the whole step against its algorithmic bytes
        achieved = round(stage_bytes * 3 * args.steps / el / 1e9, 1)
        roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": "whole RK step (graph)",
                    "alg_bytes_per_point": 3 * stage_bytes // points}
    copy_gbs = copy_bandwidth(torch)

    cfg = {"workload": wname, "blocks": nb, "points": points, "precision": args.precision, "form": form,
           "scheme": args.scheme,
           "cfl": wl.cfl, "dt": dt, "parallelism": "single GPU"}
    if nb == 1:
        cfg["grid"] = [blk.ni, blk.nj, blk.nk]
    if bt is not None:
        tc, tp = B.cfd_batch_tuning(bt)
        times = B.cfd_batch_tuning_times(bt)
        cfg["tuned_tiles"] = {"cfg": tc, "persistent": tp,
                              "candidates_ms": {f"{d}/{c}/{p}": round(v, 4) for (d, c, p), v in times.items()}}
    else:
        cfg["tiles"] = B.cfd_block_tiles(hs[0])
    out = {
        # the headline metric: updates/s is `value`, the HBM GB/s and % of peak are in `roofline`
        "metric": "grid-point RK3 stage updates/s (FP64 vs mixed/batched) + HBM GB/s % of peak",
        "value": value,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == B.CFD_FP64 else "f32+f64",
        "data": "synthetic",
        "config": cfg,
        "roofline": roofline,
        "kernels": kernels,
        "copy_GBps": round(copy_gbs, 1),
        # algorithmic bytes of whole stages over the measured time
        "step_alg_GBps": round(stage_bytes * 3 * args.steps / el / 1e9, 1),
    }
    if not args.no_cpu and nb == 1:
        out["cpu_baseline"] = cpu_baseline(wl, wname, scheme)
        one = cpu_baseline_one_thread(args.workload, scheme)
        if one is not None:
            out["cpu_baseline_1thread"] = one
    if bt is not None:
        B.cfd_batch_destroy(bt)
    B.cfd_exchange_destroy(x)
    for hb in hs:
        B.cfd_block_destroy(hb)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
