#!/usr/bin/env python3
"""Throughput of the SPH hydrodynamics step on one MI355X.

One step = one pass of the whole hot path through the C ABI (sph_step):
leapfrog predict, Morton keys, radix sort, permute, tree + groups, density
with the smoothing-length iteration, force, correct, Courant dt.  The default
workload is the largest single-GPU configuration, the turbulent box (256^3 =
16,777,216 particles, mixed FP32/FP64 pairs); the same steps are also timed
in FP64 to give the mixed/FP64 ratio, and the adjoint of one step of the same
box is timed against that step.

Prints ONE JSON line (the last line of stdout).  ``value`` is
particle-updates/s = N * steps / wall time of the timed steps, with the state
resident in HBM.  ``roofline`` is for the kernel with the longest mean launch
among the neighbour-list, density and force kernels, from its algorithmic
FLOPs and its mean launch time measured with HIP events on the library
stream (recorded on every 8th timed step); ``other_kernel_rooflines`` holds
the other two.
``cpu_baseline`` times the FP64 CPU oracle on the host cores: one full
evaluation of the workload on every core, whose fields also give the mixed
path's error per quantity against the oracle; and one thread on the same
recipe at 64^3.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "particle-updates/s (density+force, ~58 nbrs): mixed FP32/FP64 vs FP64"

# Algorithmic floating-point operations per unit of work, counted from the
# pair functions (an FMA counts 2, sqrt / rsqrt / rcp count 1), per smoothing
# kernel (M4, M6, Wendland C6):
#   force pair (r < S max(h_i,h_j)): geometry 9, r and rhat 5, v.rhat 8, two
#   kernel gradients (M4 16, M6 34, C6 28), viscosity terms 14,
#   acceleration 10, energy terms 24
FORCE_FLOPS_PER_PAIR = {0: 85, 1: 103, 2: 97}
#   density pair term per smoothing-length pass: q 1, f and f' (M4 14, M6 25,
#   C6 22), two accumulations 7
DENSITY_FLOPS_PER_PAIR_SUM = {0: 22, 1: 33, 2: 30}
#   distance test of the neighbour-list kernel: separation 3, r^2 5, list
#   radius 2 max(hl_i, h_margin h_j) 3, its square with the FP32 guard 2,
#   compare 1.  Its algorithmic work is one test per row entry (a pair within
#   the list radius); the candidates the walk's leaves bring in beyond those
#   are waste, reported as tests per row entry and per force pair.
LIST_FLOPS_PER_ENTRY = 14
#   adjoint force pair (k_adj_force, per ordered pair (k, j), both the term of
#   a_k and the mirror term of a_j): geometry and predicate 17, r and e 5,
#   w 8, F, F_r, F_h at h_k and h_j 47, viscosity speeds and T, dT/dw 24,
#   conductivity speed and its derivatives 13, brackets 9, projections 14,
#   term of k 125, mirror term 110
ADJ_FORCE_FLOPS_PER_PAIR = {0: 372, 1: 396, 2: 388}
# Vector ALU peak of the 256 CUs at 2.4 GHz for non-packed FP32 (and FP64)
# FMA: 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz.  The published FP32
# figure of 157.3 TFLOP/s needs packed FP32 instructions, which the library
# is compiled not to emit.
ALU_PEAK_TFLOPS = 78.6
PACKED_FP32_PEAK_TFLOPS = 157.3


def workload(name: str):
    from paper_1909_07439_amd import inputs

    if name == "sod":
        return inputs.sod()
    if name == "lattice":
        return inputs.lattice(32, jitter=0.05)
    if name == "kh":
        return inputs.kelvin_helmholtz(100)
    if name == "turb":
        return inputs.turbulent_box(256)
    if name == "turb64":
        return inputs.turbulent_box(64)
    if name == "blast":
        return inputs.blast_wave()
    if name == "sedov":
        return inputs.sedov()
    if name == "sod_small":
        return inputs.sod(dx_left=1.0 / 128, width=1.0 / 8)
    raise SystemExit(f"unknown workload {name}")


# phase events (HIP events at every phase boundary of sph_step) are recorded on
# one timed step in TIMING_EVERY: each recorded boundary idles the GPU for a
# few microseconds, which sampling keeps out of the throughput
TIMING_EVERY = 8


def run(cfg, precision, steps, warmup):
    import numpy as np
    import torch

    from paper_1909_07439_amd import sph

    p = sph.make_params(cfg, precision)
    parts = sph.Particles(cfg)
    ctx = sph.Context(p, cfg["n"])
    sph.sph_build_tree(ctx, parts)
    sph.sph_density(ctx, parts, want_iters=True)
    dt0 = sph.sph_force(ctx, parts, want_dt=True)
    init = parts.numpy("id", "rho", "h", "omega", "ax", "ay", "az", "dudt", "vsig_dt")
    sph.sph_set_timing(ctx, TIMING_EVERY)
    for _ in range(warmup):
        sph.sph_step(ctx, parts, 0.0)
    torch.cuda.synchronize()
    sph.sph_check(ctx)
    sph.sph_timings(ctx)  # drop the warm-up events
    st0 = sph.sph_stats(ctx)
    t0 = time.perf_counter()
    for _ in range(steps):
        sph.sph_step(ctx, parts, 0.0)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sph.sph_check(ctx)
    tim = sph.sph_timings(ctx)
    st = sph.sph_stats(ctx)
    # work per launch over exactly the timed launches
    nd = st["density_launches"] - st0["density_launches"]
    nf = st["force_launches"] - st0["force_launches"]
    nl = st["lists_launches"] - st0["lists_launches"]
    st["list_candidates_per_launch"] = \
        (st["total_list_candidates"] - st0["total_list_candidates"]) / max(nl, 1)
    st["density_pair_sums_per_launch"] = \
        (st["total_density_pair_sums"] - st0["total_density_pair_sums"]) / max(nd, 1)
    st["force_pairs_per_launch"] = (st["total_force_pairs"] - st0["total_force_pairs"]) / max(nf, 1)
    e = sph.sph_reduce(ctx, parts)
    ctx.close()
    wall = t1 - t0
    n = cfg["n"]
    order = np.argsort(init["id"])
    return dict(wall=wall, rate=n * steps / wall, ms_per_step=1e3 * wall / steps, timings=tim,
                stats=st, energy=e, init={k: v[order] for k, v in init.items()}, dt0=dt0)


KERNEL_SOURCE = os.path.join(ROOT, "paper_1909_07439_amd", "csrc", "sph_kernels.hip")


def source_digest() -> str:
    import hashlib

    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def traffic_record(kernel: str, cfg, precision: str):
    """HBM bytes per launch of ``kernel`` from the committed PMC summary for
    this workload, or None when there is none or when the kernel source has
    changed since its counters were taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{precision}_{cfg['workload']}_traffic.txt")
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        if ":" in line and not line.startswith((" ", "#")):
            k, v = line.split(":", 1)
            rec[k.strip()] = v.strip()
    if rec.get("kernel_source_sha256") != source_digest():
        return None
    try:
        return float(rec["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_calibration(mib: int):
    """A plain streaming kernel of known size for scaling the PMC byte
    counters: torch.neg over a float64 buffer reads and writes ``mib`` MiB."""
    import torch

    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    print(f"[bench] copy calibration: torch.neg over {mib} MiB in, {mib} MiB out, 3 launches",
          flush=True)


def roofline(kernel, flops, launch_ms, units, flops_per_unit, traffic):
    tf = flops / (launch_ms * 1e-3) / 1e12 if launch_ms > 0 else 0.0
    return {"kernel": kernel, "bound": "alu", "achieved": round(tf, 4), "peak": ALU_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": round(tf / ALU_PEAK_TFLOPS, 5), "traffic": traffic,
            "frac_of_packed_fp32_peak": round(tf / PACKED_FP32_PEAK_TFLOPS, 5),
            "launch_ms": round(launch_ms, 5), "units_per_launch": units,
            "flops_per_unit": flops_per_unit}


def adjoint_cost(precision, cfg=None, K=8, reps=3):
    """Cost of the gradient of a K-step rollout against the rollout itself on
    the adjoint workload (default: the 64^3 adjoint lattice): forward =
    initial evaluation + K steps, keeping the state at the start of every
    step; backward = K sph_step_adjoint calls (each replays its step, then
    runs the adjoint kernels) + the initial evaluation and its
    sph_eval_adjoint.  Median of ``reps`` repetitions."""
    import numpy as np
    import torch

    from paper_1909_07439_amd import inputs, sph

    if cfg is None:
        cfg = inputs.adjoint_lattice(64)
    p = sph.make_params(cfg, precision)
    ctx = sph.Context(p, cfg["n"])
    base = sph.Particles(cfg)
    sph.sph_build_tree(ctx, base)
    sph.sph_density(ctx, base)
    dt = sph.sph_force(ctx, base, want_dt=True)
    start = {k: torch.as_tensor(np.ascontiguousarray(cfg[k], dtype=np.float64)).cuda()
             for k in ("x", "y", "z", "vx", "vy", "vz", "m", "u", "h")}
    fw, bw = [], []
    tim = {}
    st0 = sph.sph_stats(ctx)
    for rep in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pp = sph.Particles.from_tensors(start)
        sph.sph_build_tree(ctx, pp)
        sph.sph_density(ctx, pp)
        sph.sph_force(ctx, pp)
        ckpt = []
        for _ in range(K):
            ckpt.append({k: pp.t[k].clone() for k in sph.STEP_FIELDS + ("id",)})
            sph.sph_step(ctx, pp, dt)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        g = sph.Cotangents(cfg["n"])
        g.t["ax"].fill_(1.0)
        g.t["vx"].fill_(1.0)
        if rep == 1:
            sph.sph_timings(ctx)
            st0 = sph.sph_stats(ctx)
        for s in reversed(range(K)):
            q = sph.Particles.from_tensors(ckpt[s])
            sph.sph_step_adjoint(ctx, q, dt, g)
        q = sph.Particles.from_tensors(start)
        sph.sph_build_tree(ctx, q)
        sph.sph_density(ctx, q)
        sph.sph_force(ctx, q)
        sph.sph_eval_adjoint(ctx, q, g)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        sph.sph_check(ctx)
        if rep > 0:
            fw.append(t1 - t0)
            bw.append(t2 - t1)
    tim = sph.sph_timings(ctx)
    st = sph.sph_stats(ctx)
    ctx.close()
    f, b = float(np.median(fw)), float(np.median(bw))
    # ordered force pairs per adjoint launch: force pairs of the force launches
    # in the timed backward passes (one force launch per adjoint launch)
    nf = st["force_launches"] - st0["force_launches"]
    fpl = (st["total_force_pairs"] - st0["total_force_pairs"]) / max(nf, 1)
    kk = int(cfg.get("kernel", 0))
    tag = "mixed" if precision == sph.SPH_PREC_MIXED else "fp64"
    return {"workload": cfg["workload"], "n_particles": cfg["n"], "steps": K,
            "precision": tag, "dt": dt, "forward_ms": round(1e3 * f, 3),
            "backward_ms": round(1e3 * b, 3), "backward_over_forward": round(b / f, 3),
            "adjoint_kernels_ms_per_launch": round(tim["adjoint"], 5),
            "step_forward_part_ms": round(tim["step"], 5),
            "roofline": roofline(f"k_adj_force<{tag}>", ADJ_FORCE_FLOPS_PER_PAIR[kk] * fpl,
                                 tim["adjoint_force"], {"force_pairs": fpl},
                                 ADJ_FORCE_FLOPS_PER_PAIR[kk], None)
            if tim.get("adjoint_force", 0.0) > 0 else None}


def cpu_baseline(cfg):
    """The FP64 oracle on the host cores: one full evaluation (tree, density
    iterated to the root, force) of the workload on every core, and one
    thread on the same recipe at 64^3 (a full evaluation of the big box on one
    thread would take minutes).  Returns the baseline record and the oracle's
    fields of the full evaluation (by original index)."""
    import oracle

    p = oracle.make_params(cfg)
    cores = oracle.num_threads()
    t0 = time.perf_counter()
    o = oracle.evaluate(cfg, p)
    t = time.perf_counter() - t0
    out = dict(value=cfg["n"] / t, unit="particle-updates/s", cores=cores, kind="oracle",
               sample=f"one full FP64 evaluation (tree, density iterated to the root, force) of "
                      f"the {cfg['workload']} workload, N={cfg['n']}, on {cores} threads: {t:.1f} s")
    small = workload("turb64") if cfg["workload"].startswith("turb") else None
    if small is not None:
        oracle.set_num_threads(1)
        t1 = time.perf_counter()
        oracle.evaluate(small, oracle.make_params(small))
        t1 = time.perf_counter() - t1
        oracle.set_num_threads(cores)
        out["value_1thread"] = small["n"] / t1
        out["sample_1thread"] = (f"one full FP64 evaluation of the same recipe at 64^3 "
                                 f"(N={small['n']}) on 1 thread: {t1:.1f} s")
    return out, o


def mixed_vs_oracle(init, dt0, o, c_cour):
    """Largest error of the mixed path's first evaluation against the FP64
    oracle, per quantity (h, rho, Omega relative; a and du/dt relative to the
    sum of the magnitudes of their pair terms; vsig_dt relative; the Courant
    dt relative) and the RMS of the same."""
    import numpy as np

    def rel(a, b):
        return np.abs(a - b) / np.maximum(np.abs(b), 1e-300)

    res = {}
    for k in ("h", "rho", "omega", "vsig_dt"):
        e = rel(init[k], o[k])
        res[k] = {"max": float(e.max()), "rms": float(np.sqrt(np.mean(e * e)))}
    ea = np.maximum.reduce([np.abs(init[k] - o[k]) / o["anorm"] for k in ("ax", "ay", "az")])
    eu = np.abs(init["dudt"] - o["dudt"]) / np.maximum(o["unorm"], 1e-300)
    res["a_over_anorm"] = {"max": float(ea.max()), "rms": float(np.sqrt(np.mean(ea * ea)))}
    res["dudt_over_unorm"] = {"max": float(eu.max()), "rms": float(np.sqrt(np.mean(eu * eu)))}
    res["dt"] = abs(dt0 - o["dt_next"]) / o["dt_next"]
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="turb")
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--n-group", type=int, default=None, help="particles per walk group")
    ap.add_argument("--n-leaf", type=int, default=None, help="particles per tree leaf")
    ap.add_argument("--h-margin", type=float, default=None,
                    help="neighbour-list reach in units of the support (default 1.1)")
    ap.add_argument("--kernel", default="m4", choices=["m4", "m6", "wc6"],
                    help="smoothing kernel (M4 cubic, M6 quintic, Wendland C6)")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the rollout-gradient cost on the adjoint workload")
    ap.add_argument("--adjoint-lattice", action="store_true",
                    help="measure the gradient cost of the 8-step rollout on the 64^3 adjoint "
                         "lattice instead of ONE step of the bench workload itself (the final "
                         "step of the turbulent box by default)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="after the timed steps, run a plain streaming kernel over MIB MiB "
                         "(scale for PMC byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the library has no "
              "multi-GPU path.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1909_07439_amd import sph

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    cfg = workload(args.workload)
    if args.kernel != "m4":
        from paper_1909_07439_amd import inputs

        cfg = inputs.with_kernel(cfg, args.kernel)
    if args.n_group:
        cfg["n_group"] = args.n_group
    if args.n_leaf:
        cfg["n_leaf"] = args.n_leaf
    if args.h_margin:
        cfg["h_margin"] = args.h_margin
    prec = sph.SPH_PREC_MIXED if args.precision == "mixed" else sph.SPH_PREC_FP64
    print(f"[bench] workload {cfg['workload']} n={cfg['n']} precision={args.precision} "
          f"steps={args.steps} warmup={args.warmup}", flush=True)
    main_run = run(cfg, prec, args.steps, args.warmup)
    print(f"[bench] {args.precision}: {main_run['rate']:.4e} upd/s, "
          f"{main_run['ms_per_step']:.3f} ms/step, phases {main_run['timings']}", flush=True)
    other = None
    if not args.no_fp64 and prec == sph.SPH_PREC_MIXED:
        other = run(cfg, sph.SPH_PREC_FP64, max(10, args.steps // 4), args.warmup)
        print(f"[bench] fp64: {other['rate']:.4e} upd/s, {other['ms_per_step']:.3f} ms/step, "
              f"phases {other['timings']}", flush=True)
    tim, st = main_run["timings"], main_run["stats"]
    tag = "mixed" if prec == sph.SPH_PREC_MIXED else "fp64"
    fpl, dpl = st["force_pairs_per_launch"], st["density_pair_sums_per_launch"]
    kk = int(cfg.get("kernel", 0))
    ffl, dfl = FORCE_FLOPS_PER_PAIR[kk], DENSITY_FLOPS_PER_PAIR_SUM[kk]
    lists = tim.get("lists", 0.0) > 0.0  # neighbour-list path (groups of 4 or 8)
    fname = "k_force_lists" if lists else "k_force"
    dname = "k_density_lists" if lists else "k_density"
    force = roofline(f"{fname}<{tag}>", ffl * fpl, tim["force"],
                     {"force_pairs": fpl}, ffl, traffic_record(fname, cfg, tag))
    dens = roofline(f"{dname}<{tag}>", dfl * dpl, tim["density"],
                    {"density_pair_sums": dpl}, dfl, traffic_record(dname, cfg, tag))
    kernels = [(tim["density"], dens), (tim["force"], force)]
    if lists:
        lpl = st["list_candidates_per_launch"]
        # row entries written per launch = the entries the force kernel reads
        rpl = st["force_candidates"]
        rl = roofline(f"k_lists<{tag}>", LIST_FLOPS_PER_ENTRY * rpl, tim["lists"],
                      {"row_entries": rpl}, LIST_FLOPS_PER_ENTRY,
                      traffic_record("k_lists", cfg, tag))
        rl["candidate_tests_per_row_entry"] = lpl / max(rpl, 1)
        rl["candidate_tests_per_force_pair"] = lpl / max(fpl, 1)
        kernels.append((tim["lists"], rl))
    # the dominant kernel (longest mean launch) carries the headline roofline
    kernels.sort(key=lambda kv: -kv[0])
    roof = kernels[0][1]
    others = [k for _, k in kernels[1:]]
    inter = (dpl + fpl) / (main_run["ms_per_step"] * 1e-3)
    out = {
        "metric": METRIC,
        "value": main_run["rate"],
        "unit": "particle-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_run["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if prec == sph.SPH_PREC_MIXED else "f64",
        "data": "synthetic",
        "config": {"workload": cfg["workload"], "n_particles": cfg["n"],
                   "precision": args.precision,
                   "kernel": {"m4": "M4", "m6": "M6", "wc6": "Wendland C6"}[args.kernel],
                   "hfact": cfg["hfact"],
                   "n_leaf": cfg["n_leaf"], "n_group": cfg["n_group"],
                   "h_margin": cfg.get("h_margin", 1.1)},
        "roofline": roof,
        "other_kernel_rooflines": others,
        "phase_ms": {k: round(v, 5) for k, v in tim.items()},
        "phase_events_every": TIMING_EVERY,
        "interactions_per_s": inter,
        "true_pairs_per_particle": {"density": st["density_pairs"] / cfg["n"],
                                    "force": st["force_pairs"] / cfg["n"]},
        "density_sums_per_step_max": st["max_density_sums"],
        "groups_walking_last_step": {"rows_overflow": st["groups_rows_overflow"],
                                     "h_outgrew": st["groups_h_outgrew"],
                                     "groups": st["n_groups"]},
        "candidates_per_pair": {"density": st["density_candidates"] / max(st["density_pairs"], 1),
                                "force": st["force_candidates"] / max(st["force_pairs"], 1)},
    }
    if other is not None:
        out["fp64_value"] = other["rate"]
        out["fp64_ms_per_step"] = other["ms_per_step"]
        out["mixed_over_fp64"] = main_run["rate"] / other["rate"]
        out["fp64_phase_ms"] = {k: round(v, 5) for k, v in other["timings"].items()}
        a, b = main_run["init"], other["init"]
        amag = np.sqrt(b["ax"] ** 2 + b["ay"] ** 2 + b["az"] ** 2)
        scale = max(float(np.sqrt(np.mean(amag ** 2))), 1e-300)
        out["mixed_error_vs_fp64"] = {
            "rho_max_rel": float(np.max(np.abs(a["rho"] - b["rho"]) / b["rho"])),
            "h_max_rel": float(np.max(np.abs(a["h"] - b["h"]) / b["h"])),
            "a_max_over_rms_a": float(max(np.max(np.abs(a[k] - b[k])) for k in ("ax", "ay", "az"))
                                      / scale),
        }
    if not args.no_adjoint:
        if args.adjoint_lattice:
            out["adjoint"] = adjoint_cost(prec)
        else:
            out["adjoint"] = adjoint_cost(prec, cfg=cfg, K=1, reps=2)
        print(f"[bench] adjoint: {out['adjoint']}", flush=True)
    if args.copy_calibration > 0:
        copy_calibration(args.copy_calibration)
    if not args.no_cpu_baseline:
        print("[bench] CPU oracle: one full evaluation on every host core", flush=True)
        out["cpu_baseline"], o = cpu_baseline(cfg)
        print(f"[bench] cpu_baseline {out['cpu_baseline']}", flush=True)
        if prec == sph.SPH_PREC_MIXED:
            out["mixed_error_vs_oracle"] = mixed_vs_oracle(main_run["init"], main_run["dt0"], o,
                                                           cfg["c_cour"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
