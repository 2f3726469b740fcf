#!/usr/bin/env python3
"""Throughput benchmark of the curvilinear AFWENO Navier-Stokes RK3 step on one MI355X.

A step is one full TVD-RK3 step (three fused RHS + stage evaluations and the halo
exchanges after each stage) over the whole grid.  The metric is grid-point RK3 stage
updates per second: interior points x 3 stages x steps / wall time of the timed steps.

Default workload (the largest single-GPU configuration, the one the roofline is measured
on): a 512 x 512 x 384 channel block, tanh wall stretching 2.5, bump 0.02, Mach 0.3,
Re 16200, isothermal walls, periodic in x and z, FP64, single-block launches.  The same
run adds side legs on the other throughput configurations: the channel in mixed precision,
the 256^3 Taylor-Green case in mixed precision, and the 24-block O-grid in per-block FP64
and batched mixed precision (the ratio of those two is the batched/mixed speed-up).

The headline steps are timed with the library's per-kernel event timing switched off; a
second pass of the same steps, with the HIP events on the kernels' own stream, gives each
kernel's mean launch time, from which the dominant kernel's algorithmic bandwidth is
formed (`roofline`).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
                       [--workload channel|tgv256|vortex32|ogrid24]
                       [--precision fp64|mixed] [--form single|perblock|batched]
                       [--no-cpu] [--no-legs]
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic (compulsory) HBM bytes per interior point of each kernel of the pencil
# design, by the role of a sweep in the direction order (first: no partial sum in; last:
# the RK combination).  FP64 path: Q 40 B, a metric component or J 8 B, a viscous-flux
# component 8 B.  The RK sweep reads Q^n at stages 1 and 2 only (stage 0 has Q^n = Q), so
# per launch it moves Q^n on two of three stages.
QN_AVG = 40.0 * 2.0 / 3.0
ALG_BYTES_FP64 = {
    "visc_prepass": 40 + 80 + 96,               # Q, 9 metrics + J, 12 flux planes
    "first": 40 + 24 + 32 + 40,                 # Q, 3 metrics, 4 flux planes, partial sum out
    "middle": 40 + 24 + 32 + 40 + 40,           # + partial sum in
    "last_rk": 40 + 24 + 32 + 40 + 8 + QN_AVG + 40,  # Q, metrics, fluxes, partial in, J, Qn, Qout
}
ALG_BYTES_MIXED = {
    "visc_prepass": 40 + 40 + 48,               # Q, the FP32 copy of the metrics, FP32 flux planes
    "first": 40 + 24 + 16 + 20,
    "middle": 40 + 24 + 16 + 20 + 20,
    "last_rk": 40 + 24 + 16 + 20 + 8 + QN_AVG + 40,
}
# Bytes an update must move in either precision whatever the kernel design: read Q_cur,
# the 9 metrics and J, write Q_out, and read Q^n on two of the three stages.
COMPULSORY_B = 40 + 80 + 40 + QN_AVG
DIR_NAMES = ("xi", "eta", "zeta")

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
VALU_PEAK_TFLOPS = {"fp64": 78.6, "mixed": 157.3}  # vector FP64; vector FP32 for the FP32 kernels


def kernel_bytes(table, order):
    """Algorithmic bytes per point keyed by the library's profiler names."""
    out = {"visc_prepass": table["visc_prepass"]}
    out[f"sweep_{DIR_NAMES[order[0]]}"] = table["first"]
    out[f"sweep_{DIR_NAMES[order[1]]}"] = table["middle"]
    out[f"sweep_{DIR_NAMES[order[2]]}_rk"] = table["last_rk"]
    return out


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


def load_counters(kernel: str, workload: str, precision: str):
    """Counter figures of a kernel (rocprofv3: HBM bytes per launch from FETCH_SIZE +
    WRITE_SIZE scaled by a copy kernel's reading, VALU FLOP per launch) if they were taken
    on the current kernel sources, else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path, encoding="utf-8") as fh:
            data = json.load(fh)
    except ValueError:
        return None
    ent = data.get(f"{workload}/{precision}/{kernel}")
    if not ent or ent.get("source_sha") != source_sha():
        return None
    return ent


WORKLOADS = {
    "channel": "channel_512x512x384_tanh2.5_bump0.02_mach0.3_re16200",
    "tgv256": "taylor_green_256^3_wavy_2pi_mach0.1_re1600",
    "vortex32": "isentropic_vortex_32^3_wavy_unit_mach0.5_re1000",
    "ogrid24": "o_grid_24_uneven_blocks_mach0.2_vortices_wall_farfield",
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


# ---- CPU baseline: the oracle as it stands, on a bounded sample of the workload --------
def cpu_info():
    model = None
    try:
        with open("/proc/cpuinfo", encoding="utf-8") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "cpu_count": os.cpu_count(), "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


SAMPLES = {  # (all host threads, one thread) instances of each workload, same per-point work
    "channel": ((256, 256, 96), (128, 128, 32)),
    "tgv256": ((128, 128, 128), (64, 64, 64)),
    "vortex32": ((32, 32, 32), (32, 32, 32)),
}


def _sample_workload(name, shape):
    from paper_2006_07964_amd import workloads as W
    if name == "channel":
        return W.channel(*shape)
    if name == "tgv256":
        return W.taylor_green_wavy(shape[0])
    return W.vortex_wavy(shape[0])


CPU_SECONDS = 10.0  # the oracle's timed sample lasts at least this long
CPU_MAX_STEPS = 8


def cpu_baseline(workload: str, scheme: int, threads: int = 0):
    """Full RK3 steps (three stages with halo fills) of a smaller instance of the same
    workload, same scheme and boundary conditions, same arithmetic per point, repeated until
    at least CPU_SECONDS have passed (at most CPU_MAX_STEPS steps).  threads = 0: every OpenMP
    thread the oracle has; 1: one thread (the paper quotes one CPU core)."""
    import oracle as O
    if workload not in SAMPLES:
        return None
    shape = SAMPLES[workload][0 if threads == 0 else 1]
    wl = _sample_workload(workload, shape)
    b = wl.blocks[0]
    c = O.cfg_from_workload(wl, scheme=scheme)
    met = O.metrics(c, b.xyz)
    dt = O.dt_cfl(c, met, b.q, wl.cfl)
    before = O.set_threads(threads) if threads else None
    try:
        used = O.threads()
        q, steps = b.q, 0
        t0 = time.perf_counter()
        while steps < CPU_MAX_STEPS and (steps == 0 or time.perf_counter() - t0 < CPU_SECONDS):
            q = O.rk_step(c, met, dt, q)
            steps += 1
        el = time.perf_counter() - t0
    finally:
        if before is not None:
            O.set_threads(before)
    out = {"value": 3 * b.points * steps / el, "unit": "updates/s", "cores": used, "kind": "oracle",
           "sample": f"{steps} RK3 step(s) (3 stages each: RHS, update, halo fill) of the {b.ni}x{b.nj}x{b.nk} "
                     f"instance of the {workload} workload, {el:.2f} s on {used} OpenMP thread(s)"}
    out.update(cpu_info())
    return out


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


# ---- one measured configuration ------------------------------------------------------
def run_leg(torch, B, wl, wname, precision, form, steps, warmup, scheme=0, tiles=None, profile_steps=0):
    """Set the workload up on the device, run `warmup` untimed steps and `steps` timed ones
    (library event timing off), then, if profile_steps > 0, that many more with the
    per-kernel HIP events on.  Returns a dict; frees every device buffer it made."""
    prec = B.CFD_FP64 if precision == "fp64" else B.CFD_MIXED
    stream = torch.cuda.current_stream()
    nb = len(wl.blocks)
    form = form or ("single" if nb == 1 else "perblock")
    if form == "single" and nb != 1:
        raise SystemExit("--form single needs a single-block workload")
    hs, qs, qas, qbs = [], [], [], []
    for bi, blk in enumerate(wl.blocks):
        # rows padded to 16 doubles and offset so that interior rows start 128-byte lines
        desc = B.desc_from_workload(wl, bi, prec, ld_i=B.aligned_pitch(blk.ni), scheme=scheme)
        h = B.cfd_block_create(desc, stream)
        if tiles:
            B.cfd_block_set_tiles(h, tiles)
        xyz = torch.from_numpy(blk.xyz).cuda()
        B.cfd_metrics(h, xyz, blk.ni + 12, blk.nj + 12)
        del xyz
        hs.append(h)
        qs.append(B.upload_state(desc, blk.q))
        qas.append(B.upload_state(desc, blk.q))
        qbs.append(B.upload_state(desc, blk.q))
    x = B.cfd_exchange_create(hs, wl.interfaces)
    B.cfd_halo_exchange(x, B.CFD_FIELDS_Q, qs)
    dt = B.cfd_dt_cfl(hs, qs, wl.cfl)
    dt_dev = torch.tensor([dt], dtype=torch.float64, device="cuda")
    points = wl.points
    bt = B.cfd_batch_create(hs, x, stream) if form == "batched" else None
    h, q, qa, qb = hs[0], qs[0], qas[0], qbs[0]

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

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    res = {"workload": wname, "precision": precision, "form": form, "blocks": nb, "points": points,
           "steps": steps, "warmup": warmup, "dt": dt, "cfl": wl.cfl,
           "value": points * 3 * steps / el, "ms_per_step": el / steps * 1e3}
    if nb == 1:
        res["grid"] = [wl.blocks[0].ni, wl.blocks[0].nj, wl.blocks[0].nk]
    if bt is not None:
        tc, tp = B.cfd_batch_tuning(bt)
        res["tuned_tiles"] = {"cfg": tc, "persistent": tp}
    else:
        res["tiles"] = B.cfd_block_tiles(hs[0])
    if profile_steps > 0 and form != "batched":
        for hb in hs:
            B.cfd_profile_reset(hb)
            B.cfd_profile_enable(hb, True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(profile_steps):
            step()
        torch.cuda.synchronize()
        elp = time.perf_counter() - t0
        prof = {}
        for hb in hs:
            B.cfd_profile_enable(hb, False)
            for name, (launches, ms) in B.cfd_profile_read(hb).items():
                l0, m0 = prof.get(name, (0, 0.0))
                prof[name] = (l0 + launches, m0 + ms)
        res["prof"] = prof
        res["profiled_value"] = points * 3 * profile_steps / elp
        res["profile_steps"] = profile_steps
    for hb, qb_ in zip(hs, qs):
        if not B.cfd_check_finite(hb, qb_):
            raise SystemExit(f"non-finite state after the timed steps of {wname} ({precision}, {form})")
    if bt is not None:
        B.cfd_batch_destroy(bt)
    B.cfd_exchange_destroy(x)
    for hb in hs:
        B.cfd_block_destroy(hb)
    del qs, qas, qbs, q, qa, qb, dt_dev
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return res


def kernel_table(res, B, workload_key):
    """Per-kernel mean launch time and algorithmic bandwidth from a profiled leg, and the
    roofline entry of the dominant kernel (largest total time)."""
    prec = res["precision"]
    alg = kernel_bytes(ALG_BYTES_FP64 if prec == "fp64" else ALG_BYTES_MIXED, B.cfd_sweep_order())
    prof, points, nb = res["prof"], res["points"], res["blocks"]
    kernels = {}
    total_ms = sum(v[1] for v in prof.values())
    for name, (launches, ms) in prof.items():
        ent = {"launches": launches, "avg_ms": round(ms / max(launches, 1), 4), "share": round(ms / total_ms, 3)}
        if name in alg:
            total_bytes = alg[name] * points * launches / nb  # every block launches each kernel equally often
            ent["alg_bytes_per_launch"] = int(total_bytes / launches)
            ent["alg_GBps"] = round(total_bytes / (ms * 1e-3) / 1e9, 1)
            ent["alg_frac"] = round(total_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
            cnt = load_counters(name, workload_key, prec)
            if cnt and cnt.get("flop_per_launch"):
                tf = cnt["flop_per_launch"] * launches / (ms * 1e-3) / 1e12
                ent["valu_TFLOPs"] = round(tf, 2)
                ent["valu_frac"] = round(tf / VALU_PEAK_TFLOPS[prec], 4)
        kernels[name] = ent
    dom = max((n for n in kernels if n in alg), key=lambda n: prof[n][1])
    dk = kernels[dom]
    cnt = load_counters(dom, workload_key, prec)
    roofline = {"bound": "hbm", "achieved": dk["alg_GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": dk["alg_frac"], "traffic": cnt.get("bytes_per_launch") if cnt else None,
                "kernel": dom, "alg_bytes_per_point": round(alg[dom], 2),
                "points_per_launch": points // nb, "avg_launch_ms": dk["avg_ms"]}
    return kernels, roofline, alg


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="channel", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--form", default=None, choices=["single", "perblock", "batched"],
                    help="single-block calls, per-block launches, or the batched graph form")
    ap.add_argument("--profile-steps", type=int, default=5,
                    help="steps of the second pass with per-kernel event timing")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--no-legs", action="store_true", help="skip the side legs of the default run")
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
    scheme = B.CFD_AFWENO_ORIGINAL if args.scheme == "original" else B.CFD_AFWENO_MODIFIED
    tiles = [int(v) for v in args.tiles.split(",")] if args.tiles else None
    t_start = time.perf_counter()
    wl, wname = build_workload(args.workload)
    head = run_leg(torch, B, wl, wname, args.precision, args.form, args.steps, args.warmup, scheme, tiles,
                   profile_steps=args.profile_steps)
    print(f"# headline {wname} {args.precision} {head['form']}: {head['value']:.4g} updates/s "
          f"({time.perf_counter() - t_start:.0f} s)", file=sys.stderr, flush=True)

    value = head["value"]
    cfg = {k: head[k] for k in ("workload", "blocks", "points", "precision", "form", "cfl", "dt") if k in head}
    cfg.update({"scheme": args.scheme, "parallelism": "single GPU"})
    for k in ("grid", "tiles", "tuned_tiles"):
        if k in head:
            cfg[k] = head[k]
    out = {
        # the headline metric: updates/s is `value`, the HBM GB/s and % of peak are in `roofline`
        "metric": "grid-point RK3 stage updates/s (FP64 vs mixed/batched) + HBM GB/s % of peak",
        "value": value,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": cfg,
    }
    design_bytes = None
    if "prof" in head:
        kernels, roofline, alg = kernel_table(head, B, args.workload)
        out["roofline"] = roofline
        out["kernels"] = kernels
        out["profiled_pass"] = {"steps": head["profile_steps"], "value": head["profiled_value"]}
        design_bytes = sum(alg.values())
    copy_gbs = copy_bandwidth(torch)
    hbm = {"copy_GBps": round(copy_gbs, 1), "copy_frac": round(copy_gbs / HBM_PEAK_GBS, 4),
           "compulsory_B_per_update": round(COMPULSORY_B, 2),
           "compulsory_GBps": round(COMPULSORY_B * value / 1e9, 1),
           "compulsory_frac": round(COMPULSORY_B * value / 1e9 / HBM_PEAK_GBS, 4)}
    if design_bytes is not None:
        # the pencil design's algorithmic bytes of whole stages over the timed steps
        hbm["design_B_per_update"] = round(design_bytes, 2)
        hbm["step_alg_GBps"] = round(design_bytes * value / 1e9, 1)
        hbm["step_alg_frac"] = round(design_bytes * value / 1e9 / HBM_PEAK_GBS, 4)
        # binding roof of the step: the larger of its HBM and VALU fractions (VALU from the
        # counter figures of the current sources, when present)
        k = out["kernels"]
        if all("valu_frac" in k[n] for n in alg if n in k):
            tot_ms = sum(k[n]["avg_ms"] * k[n]["launches"] for n in alg if n in k)
            vf = sum(k[n]["valu_frac"] * k[n]["avg_ms"] * k[n]["launches"] for n in alg if n in k) / tot_ms
            hbm["step_valu_frac"] = round(vf, 4)
            hbm["binding_frac"] = round(max(vf, hbm["step_alg_frac"]), 4)
    out["hbm"] = hbm

    # ---- side legs of the default run: the other throughput configurations ------------
    if not args.no_legs and args.workload == "channel" and args.precision == "fp64" and head["form"] == "single":
        legs = {}
        res = run_leg(torch, B, wl, wname, "mixed", "single", args.steps, args.warmup, scheme)
        legs["channel_mixed_single"] = {"value": res["value"], "ms_per_step": res["ms_per_step"]}
        del wl
        print(f"# channel mixed: {res['value']:.4g} updates/s ({time.perf_counter() - t_start:.0f} s)",
              file=sys.stderr, flush=True)
        wl3, n3 = build_workload("tgv256")
        res = run_leg(torch, B, wl3, n3, "mixed", "single", 20, 3, scheme)
        legs["tgv256_mixed_single"] = {"workload": n3, "value": res["value"], "ms_per_step": res["ms_per_step"]}
        del wl3
        print(f"# tgv256 mixed: {res['value']:.4g} updates/s ({time.perf_counter() - t_start:.0f} s)",
              file=sys.stderr, flush=True)
        wl4, n4 = build_workload("ogrid24")
        r64 = run_leg(torch, B, wl4, n4, "fp64", "perblock", 10, 3, scheme)
        rmx = run_leg(torch, B, wl4, n4, "mixed", "batched", 10, 3, scheme)
        del wl4
        legs["ogrid24_fp64_perblock"] = {"workload": n4, "value": r64["value"], "ms_per_step": r64["ms_per_step"]}
        legs["ogrid24_mixed_batched"] = {"workload": n4, "value": rmx["value"], "ms_per_step": rmx["ms_per_step"],
                                         "tuned_tiles": rmx.get("tuned_tiles")}
        legs["ogrid24_batched_mixed_over_perblock_fp64"] = round(rmx["value"] / r64["value"], 3)
        print(f"# ogrid24: fp64 per-block {r64['value']:.4g}, mixed batched {rmx['value']:.4g} "
              f"({time.perf_counter() - t_start:.0f} s)", file=sys.stderr, flush=True)
        out["legs"] = legs

    if not args.no_cpu and args.workload in SAMPLES:
        out["cpu_baseline"] = cpu_baseline(args.workload, scheme, threads=0)
        one = cpu_baseline(args.workload, scheme, threads=1)
        if one is not None:
            out["cpu_baseline_1thread"] = one
    out["bench_wall_s"] = round(time.perf_counter() - t_start, 1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
