#!/usr/bin/env python3
"""Benchmark: solves/s to relative residual 1e-10 on the 4097 x 4097 vertex
heterogeneous diffusion problem (-div(D grad u) = f, zero Dirichlet data,
5-point finite volumes, D piecewise constant on 16 x 16-cell blocks with
log10 D ~ U[-2, 2]), V(2,1) cycles, FP64; plus FP32 V-cycles inside FP64
iterative refinement on the same operator and on a two-phase checkerboard.

A step is one complete solve from u = 0 to ||b - A u|| / ||b|| <= 1e-10 with
the hierarchy already built and the inputs resident in HBM (the paper times
the solve phase; setup is reported separately).

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
TOL = 1e-10


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def stream_source_sha():
    with open(os.path.join(ROOT, "paper_1803_02481_amd", "csrc", "bmg_stream.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        t = json.load(open(path))
    except ValueError:
        return None
    if t.get("source_sha") != stream_source_sha() or t.get("kernel") != kernel:
        return None
    return t.get("hbm_bytes_per_launch")


def measured_traffic3d():
    """HBM bytes of one 3D finest relaxation sweep from the committed counter
    summary, if it was taken on the current 3D source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic3d.json")
    if not os.path.exists(path):
        return None
    try:
        t = json.load(open(path))
    except ValueError:
        return None
    with open(os.path.join(ROOT, "paper_1803_02481_amd", "csrc", "bmg3d.hip"), "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()[:16]
    if t.get("source_sha") != sha:
        return None
    return t.get("sweep_hbm_bytes")


def time_solves(hier, b, steps, warmup, torch):
    u = torch.zeros_like(b)
    info = None
    for _ in range(warmup):
        u.zero_()
        u, info = hier.solve(b, u, tol=TOL)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        u.zero_()
        u, info = hier.solve(b, u, tol=TOL)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    return el, u, info


def per_cycle(HB, torch, coeffs, b, reps=3, **prm):
    """Seconds per V-cycle of a configuration: a 12-cycle solve minus a
    6-cycle solve (what every solve pays once drops out), median of `reps`
    such differences; and the model's time for the configuration (us)."""
    hs = {kc: HB.Hierarchy(coeffs, max_cycles=kc, **prm) for kc in (6, 12)}
    for h in hs.values():
        h.solve(b, tol=1e-30, check=False)
    diffs, model = [], 0.0
    for _ in range(reps):
        tk = {}
        for kc, h in hs.items():
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, info = h.solve(b, tol=1e-30, check=False)
            torch.cuda.synchronize()
            tk[kc] = time.perf_counter() - t0
            model = info.path_us
        diffs.append((tk[12] - tk[6]) / 6.0)
    del hs
    return sorted(diffs)[len(diffs) // 2], model


def host_info():
    """The host the oracle runs on: CPU model, logical CPUs, the CPUs this
    process may use, and OMP_NUM_THREADS."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return {"cpu_model": model, "os_cpu_count": os.cpu_count(), "usable_cpus": usable,
            "OMP_NUM_THREADS": os.environ.get("OMP_NUM_THREADS")}


def oracle_threads():
    """Threads for the all-core oracle runs: OMP_NUM_THREADS if set (the share
    of the host this process is given), else every CPU it may use."""
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) >= 1:
        return int(env)
    return host_info()["usable_cpus"] or 1


def oracle_workloads(args, n, extra, O, np, inputs):
    """The FP64 oracle, on all the host cores this process is given, timed on
    bounded samples of the other workloads (its FP32 mode emulates the inner
    solver for checking; every entry here is an FP64 solve)."""
    res = {}
    nth = oracle_threads()
    O.set_threads(nth)
    # 65^2, D = 1: the whole solve
    m = 65
    oh = O.Hierarchy(O.fv5(inputs.cells_constant(m, m)))
    bm = inputs.load_uniform(m, m, seed=0)
    t0 = time.perf_counter()
    _, hist = oh.solve(bm, tol=TOL)
    el = time.perf_counter() - t0
    res["constant_65"] = {"value": 1.0 / el, "unit": "solves/s", "cores": nth,
                          "sample": "whole FP64 solve, %d cycles" % (len(hist))}
    # two-phase checkerboard at n^2: a few cycles, scaled by the GPU solve's
    # FP64 cycle count
    cb = extra.get("checkerboard", {}).get("fp64")
    if cb:
        oh = O.Hierarchy(O.fv5(inputs.cells_two_phase_blocks(n, n, 64, (1.0, 1e-3), seed=3)))
        bc = inputs.load_uniform(n, n, seed=4)
        uc = np.zeros_like(bc)
        k = max(1, args.cpu_cycles // 2)
        t0 = time.perf_counter()
        for _ in range(k):
            uc = oh.vcycle(bc, uc)
        tc = (time.perf_counter() - t0) / k
        res["checkerboard_%d" % n] = {"value": 1.0 / (tc * cb["cycles"]), "unit": "solves/s", "cores": nth,
                                      "sample": "%d FP64 cycles (%.2f s/cycle), scaled by the %d cycles of the "
                                                "GPU FP64 solve" % (k, tc, cb["cycles"])}
        del oh
    # the paper's workload: a few cycles at full size, scaled to its 10
    if "paper_workload" in extra:
        px, py = 16385, 1025
        Dxp, Dyp = inputs.cells_compensating(px, py)
        hx, hy = inputs.spacings(px, py)
        oh = O.Hierarchy(O.fv5_aniso(Dxp, Dyp, hx, hy))
        bp = inputs.load_uniform(px, py, seed=12)
        up = np.zeros_like(bp)
        k = max(1, args.cpu_cycles // 2)
        t0 = time.perf_counter()
        for _ in range(k):
            up = oh.vcycle(bp, up)
        tc = (time.perf_counter() - t0) / k
        res["paper_workload"] = {"value": 1e3 * 10 * tc, "unit": "ms per 10 cycles", "cores": nth,
                                 "sample": "%d FP64 cycles (%.2f s/cycle), scaled to 10" % (k, tc)}
        del oh
    # batched: the first 8 problems solved whole, scaled to the batch by vertex count
    if "batched" in extra:
        sizes = inputs.batch_sizes(args.batch, seed=5)
        sample = list(range(min(8, len(sizes))))
        t_s, pts = 0.0, 0
        for i in sample:
            mi = sizes[i]
            oh = O.Hierarchy(O.fv5(inputs.cells_lognormal(mi, mi, 1.0, seed=1000 + i)))
            bi = inputs.load_uniform(mi, mi, seed=2000 + i)
            t0 = time.perf_counter()
            oh.solve(bi, tol=TOL)
            t_s += time.perf_counter() - t0
            pts += mi * mi
            del oh
        t_batch = t_s * extra["batched"]["points"] / pts
        res["batched"] = {"value": len(sizes) / t_batch, "unit": "problems/s", "cores": nth,
                          "sample": "FP64 solves of problems 0-%d (sizes %s, %.2f s), scaled to the batch's "
                                    "%d vertices" % (len(sample) - 1, [sizes[i] for i in sample], t_s,
                                                     extra["batched"]["points"])}
    # adjoint: one 1025^2 gradient (forward solve, adjoint solve, cell kernel)
    if "adjoint" in extra:
        m = 1025
        theta = inputs.theta_box5(m, m, seed=3000)
        ba = inputs.load_uniform(m, m, seed=5000)
        u_obs, _ = O.Hierarchy(O.fv5(np.exp(inputs.theta_box5(m, m, seed=4000)))).solve(ba, tol=TOL)
        t0 = time.perf_counter()
        D = np.exp(theta)
        oh = O.Hierarchy(O.fv5(D))
        uo, _ = oh.solve(ba, tol=TOL)
        lam, _ = oh.solve(uo - u_obs, tol=TOL)
        O.grad_logD(D, uo, lam)
        el = time.perf_counter() - t0
        res["adjoint"] = {"value": 1.0 / el, "unit": "gradients/s", "cores": nth,
                          "sample": "one %dx%d gradient: setup, FP64 forward and adjoint solves, cell kernel "
                                    "(%.2f s)" % (m, m, el)}
    # 3D: two V-cycles of the 3D oracle at 129^3 (its 257^3 setup alone takes
    # minutes), scaled by vertex count to 257^3 and by the cycles of the GPU
    # solve
    if "next_3d" in extra:
        m = 129
        oh = O.Hierarchy3(O.fv7(inputs.cells3_log10_blocks(m, m, m, block=8, seed=51)))
        bm = inputs.load3_uniform(m, m, m, seed=53)
        um = np.zeros_like(bm)
        k = 2
        t0 = time.perf_counter()
        for _ in range(k):
            um = oh.vcycle(bm, um)
        tc = (time.perf_counter() - t0) / k
        n3 = extra["next_3d"]["n"]
        scale = (n3 / m) ** 3
        cyc = extra["next_3d"]["cycles"]
        res["next_3d"] = {"value": 1.0 / (tc * scale * cyc), "unit": "solves/s", "cores": nth,
                          "sample": "%d FP64 V(2,1)-cycles of the 3D oracle at %d^3 (%.3f s/cycle), scaled by "
                                    "vertex count to %d^3 and by the %d cycles of the GPU solve"
                                    % (k, m, tc, n3, cyc)}
        del oh
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=4097)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-cycles", type=int, default=4, help="oracle V-cycles timed for the baseline")
    ap.add_argument("--cpu-solve-max-s", type=float, default=40.0,
                    help="time the oracle's whole solve when the timed cycles say it takes at most this long")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--collapse-level", type=int, default=-1)
    ap.add_argument("--no-paper", action="store_true", help="skip the paper's own workload")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched workload")
    ap.add_argument("--batch", type=int, default=256, help="problems in the batched workload")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the batched adjoint workload")
    ap.add_argument("--adjoint-batch", type=int, default=64, help="problems in the adjoint workload")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip timing each forced collapse level against the model")
    ap.add_argument("--no-3d", action="store_true", help="skip the 3D workload")
    ap.add_argument("--n3", type=int, default=257, help="vertices per side of the 3D workload")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1803_02481_amd import hipbmg as HB
    from paper_1803_02481_amd import inputs

    dev = "cuda:0"
    n = args.n
    log("bench: building inputs n=%d" % n)
    D = torch.from_numpy(inputs.cells_log10_blocks(n, n, 16, -2.0, 2.0, seed=1)).to(dev)
    b = torch.from_numpy(inputs.load_uniform(n, n, seed=2)).to(dev)
    coeffs = HB.fv5_from_cells(D)
    torch.cuda.synchronize()

    log("bench: calibrating the collapse-level model")
    calib = HB.calibrate()
    log("bench: calibration %s" % {k: round(v, 3) for k, v in calib.items()})
    log("bench: FP64 setup")
    hier = HB.Hierarchy(coeffs, collapse_level=args.collapse_level)
    _, info0 = hier.solve(b, tol=TOL)          # also a warm-up
    hier.profile(True)
    log("bench: FP64 timed solves (%d)" % args.steps)
    el, u64, info = time_solves(hier, b, args.steps, args.warmup, torch)
    hier.profile(False)
    prof = hier.profile_read(0)
    ms_per_step = 1e3 * el / args.steps
    value = args.steps / el
    cycles = info.cycles
    # dominant kernel: largest summed time over the timed solves
    kname, (kms, kn, kbytes) = max(prof.items(), key=lambda kv: kv[1][0])
    kavg_s = kms / kn / 1e3
    achieved = kbytes / kavg_s / 1e9
    traffic = measured_traffic(kname)
    kernels = {k: {"avg_us": 1e3 * v[0] / v[1], "launches": v[1],
                   "GBps": v[2] / (v[0] / v[1] / 1e3) / 1e9} for k, v in prof.items()}
    log("bench: FP64 %.3f solves/s, %d cycles, %.3f ms/solve, dominant %s %.1f GB/s"
        % (value, cycles, ms_per_step, kname, achieved))

    extra = {}
    # per-level table: one more solve with every level's kernels timed, next
    # to the model's terms for the same levels
    hier.profile(True, levels=True)
    _, info_l = hier.solve(b, tol=TOL)
    hier.profile(False)
    lv_ms = hier.profile_levels(0)
    mod = hier.model_levels()
    ls_ = info_l.collapse_level
    table = []
    for l in range(info_l.levels):
        ny_l, nx_l = hier.size(l)
        row = {"level": l, "n": nx_l}
        if l > ls_:
            row.update(mode="grid", measured_us_per_cycle=1e3 * (lv_ms[l][0] + lv_ms[l][1]) / info_l.cycles,
                       model_us_per_cycle=mod["grid_us"][l])
        elif l == ls_:
            row.update(mode="collapse launch (levels 0..%d)" % ls_,
                       measured_us_per_cycle=1e3 * lv_ms[l][2] / info_l.cycles,
                       model_us_per_cycle=mod["base_us"] + sum(mod["collapsed_us"][1: ls_ + 1]))
        else:
            continue
        table.append(row)
    extra["levels_fp64"] = table
    log("bench: per-level " + ", ".join("%d:%.0f/%.0f" % (r["n"], r["measured_us_per_cycle"], r["model_us_per_cycle"])
                                        for r in table))
    if not args.no_sweep:
        # every forced collapse level l*: measured time per V-cycle next to the
        # model's prediction (the one-GPU form of the paper's path comparison)
        sweep = []
        model = list(info.model_us)[: info.levels]
        for ls in range(0, info.levels):
            if model[ls] > 20 * min(model):
                continue
            # per cycle from a 12-cycle and a 6-cycle solve: the difference
            # leaves out what every solve pays once (first pre-relaxations,
            # ||b||, copies)
            per, _ = per_cycle(HB, torch, coeffs, b, collapse_level=ls)
            sweep.append({"collapse_level": ls, "measured_us_per_cycle": 1e6 * per,
                          "model_us_per_cycle": model[ls]})
            log("bench: l*=%d measured %.1f us/cycle, model %.1f" % (ls, 1e6 * per, model[ls]))
        extra["collapse_sweep"] = sweep
        # forced agglomeration stages above the model's l*: one stage of K
        # workgroups on the next one or two levels, measured against the
        # model's time for that configuration (the search's alternatives)
        ssweep = []
        ls0 = info.collapse_level
        for top in (ls0 + 1, ls0 + 2):
            if top > info.levels - 2:
                continue
            for wg in (2, 16, 256):
                per, pus = per_cycle(HB, torch, coeffs, b, collapse_level=ls0, cluster_wg=wg, cluster_top=top)
                ssweep.append({"collapse_level": ls0, "stage_workgroups": wg, "stage_top": top,
                               "measured_us_per_cycle": 1e6 * per, "model_us_per_cycle": pus})
                log("bench: stage of %d workgroups on levels %d..%d above l*=%d: measured %.1f us/cycle, model %.1f"
                    % (wg, top, ls0 + 1, ls0, 1e6 * per, pus))
        extra["stage_sweep"] = ssweep
        # coarsest grid size: coarsening stops at the first level with a side
        # <= coarsest_n, solved with its dense Cholesky factor (section 3's
        # coarse-solve term grows as the square of its unknowns); cycles to the
        # tolerance and time per solve for each size
        csweep = []
        for cn in (3, 5, 9, 17, 33):
            hc = HB.Hierarchy(coeffs, coarsest_n=cn)
            el_c, _, info_c = time_solves(hc, b, 3, 1, torch)
            csweep.append({"coarsest_n": cn, "levels": info_c.levels, "cycles": info_c.cycles,
                           "ms_per_solve": 1e3 * el_c / 3, "us_per_cycle": 1e6 * el_c / 3 / info_c.cycles,
                           "collapse_level": info_c.collapse_level, "relres": info_c.relres})
            log("bench: coarsest_n %d: %d levels, %d cycles, %.2f ms/solve" % (cn, info_c.levels, info_c.cycles,
                                                                             1e3 * el_c / 3))
            hc.close()
        extra["coarsest_sweep"] = csweep
        best = min(sweep, key=lambda r: r["measured_us_per_cycle"])
        chosen = [r for r in sweep if r["collapse_level"] == info.collapse_level]
        if chosen:
            extra["collapse_choice"] = {
                "model": info.collapse_level, "measured_best": best["collapse_level"],
                "model_choice_over_best": chosen[0]["measured_us_per_cycle"] / best["measured_us_per_cycle"]}
    if not args.no_mixed:
        log("bench: mixed precision on the same operator")
        hm = HB.Hierarchy(coeffs, precision=HB.MIXED, collapse_level=args.collapse_level)
        hm.solve(b, tol=TOL)
        el_m, um, infom = time_solves(hm, b, args.steps, args.warmup, torch)
        err = float((um - u64).abs().max() / u64.abs().max())
        extra["mixed_blocks"] = {"solves_per_s": args.steps / el_m, "ms_per_solve": 1e3 * el_m / args.steps,
                                 "fp32_cycles": infom.cycles, "refinement_steps": infom.outer_steps,
                                 "relres": infom.relres, "max_rel_diff_vs_fp64": err}
        log("bench: mixed %.3f solves/s (%d FP32 cycles, %d steps)"
            % (args.steps / el_m, infom.cycles, infom.outer_steps))
        del hm
        # the two-phase checkerboard operator, FP64 and mixed
        Dc = torch.from_numpy(inputs.cells_two_phase_blocks(n, n, 64, (1.0, 1e-3), seed=3)).to(dev)
        bc = torch.from_numpy(inputs.load_uniform(n, n, seed=4)).to(dev)
        cc = HB.fv5_from_cells(Dc)
        res = {}
        for name, prec in (("fp64", HB.FP64), ("mixed", HB.MIXED)):
            hc = HB.Hierarchy(cc, precision=prec, collapse_level=args.collapse_level)
            hc.solve(bc, tol=TOL)
            el_c, uc, infoc = time_solves(hc, bc, args.steps, args.warmup, torch)
            res[name] = {"solves_per_s": args.steps / el_c, "ms_per_solve": 1e3 * el_c / args.steps,
                         "cycles": infoc.cycles, "refinement_steps": infoc.outer_steps,
                         "relres": infoc.relres}
            res[name + "_u"] = uc
            del hc
            log("bench: checkerboard %s %.3f solves/s" % (name, args.steps / el_c))
        res["max_rel_diff_mixed_vs_fp64"] = float((res["mixed_u"] - res["fp64_u"]).abs().max()
                                                  / res["fp64_u"].abs().max())
        del res["mixed_u"], res["fp64_u"]
        extra["checkerboard"] = res

    if not args.no_paper:
        # the paper's own workload (section 5): the unit square on a stretched
        # 16385 x 1025 vertex grid (16:1, a 2:1 processor grid of 8:1 local
        # problems, as one GPU's share), D = diag(1/r, r) with r = hy/hx = 16,
        # f ~ U[-1,1], and a fixed 10 V(2,1)-cycles from zero, as its runs time
        px, py = 16385, 1025
        log("bench: paper workload %dx%d, 10 V(2,1)-cycles" % (px, py))
        Dxp, Dyp = inputs.cells_compensating(px, py)
        hx, hy = inputs.spacings(px, py)
        cp = HB.fv5_aniso(torch.from_numpy(Dxp).to(dev), torch.from_numpy(Dyp).to(dev), hx, hy)
        bp = torch.from_numpy(inputs.load_uniform(px, py, seed=12)).to(dev)
        hp = HB.Hierarchy(cp, max_cycles=10)
        up, ip = hp.solve(bp, tol=1e-30, check=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            up, ip = hp.solve(bp, tol=1e-30, check=False)
        torch.cuda.synchronize()
        el_p = (time.perf_counter() - t0) / args.steps
        hist = ip.history()
        extra["paper_workload"] = {
            "workload": "%dx%d vertices on the unit square (hx/hy = 1/16), D = diag(1/16, 16) per cell, f ~ "
                        "U[-1,1] (seed 12), 10 V(2,1)-cycles from zero, FP64" % (px, py),
            "ms_per_10_cycles": 1e3 * el_p,
            "us_per_cycle": 1e6 * el_p / 10,
            "relres_after_10": hist[-1],
            "rate_per_cycle": (hist[-1] / hist[0]) ** (1.0 / 9),
            "levels": ip.levels, "collapse_level": ip.collapse_level, "stages": ip.cluster_stages,
        }
        log("bench: paper workload %.2f ms per 10 cycles, relres %.2e, rate %.3f"
            % (1e3 * el_p, hist[-1], extra["paper_workload"]["rate_per_cycle"]))
        del hp, cp, bp, up
        # the paper's redistribution search in its own form (section 4), weak
        # scaling of its search-time figure: local 568 x 71 on 2:1 processor
        # grids, the paper's machine parameters; host only
        scal = []
        for k in range(1, 16):
            P = (2 ** ((k + 1) // 2), 2 ** (k // 2))
            N = (568 * P[0], 71 * P[1])
            reps = 20
            t0 = time.perf_counter()
            for _ in range(reps):
                t_ex, _ = HB.paper_search(N, P)
            t_exh = (time.perf_counter() - t0) / reps
            t0 = time.perf_counter()
            for _ in range(reps):
                t_as, path, expanded = HB.paper_astar(N, P)
            t_ast = (time.perf_counter() - t0) / reps
            scal.append({"n_p": P[0] * P[1], "processor_grid": list(P), "brute_force_paths": P[0] * P[1] // 2,
                         "astar_expanded": expanded, "path_length": len(path),
                         "astar_us": 1e6 * t_ast, "exhaustive_us": 1e6 * t_exh,
                         "model_s_per_cycle": t_as, "same_optimum": abs(t_as - t_ex) <= 1e-12 * t_ex})
        extra["paper_search_scaling"] = scal

    if not args.no_batch:
        # many independent problems of different sizes in one batched solve:
        # sizes from {129, 257, 513, 1025}^2, per-cell lognormal D (sigma 1),
        # FP32 V-cycles inside FP64 refinement, one cycle replayed as a graph
        log("bench: batched workload (%d problems)" % args.batch)
        sizes = inputs.batch_sizes(args.batch, seed=5)
        cs, bs = [], []
        for i, m in enumerate(sizes):
            Di = torch.from_numpy(inputs.cells_lognormal(m, m, 1.0, seed=1000 + i)).to(dev)
            cs.append(HB.fv5_from_cells(Di))
            bs.append(torch.from_numpy(inputs.load_uniform(m, m, seed=2000 + i)).to(dev))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bh = HB.BatchHierarchy(cs, precision=HB.MIXED)
        t_setup = time.perf_counter() - t0
        us = [torch.zeros_like(x) for x in bs]
        bh.solve(bs, us, tol=TOL)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            for x in us:
                x.zero_()
            us, infos_b = bh.solve(bs, us, tol=TOL)
        torch.cuda.synchronize()
        el_b = time.perf_counter() - t0
        npts = sum(m * m for m in sizes)
        # the tile shape the autotuner chose: strips per workgroup, the cap on
        # row-pair steps per tile, and each size's row blocks, finest level first
        shape = {}
        for m in sorted(set(sizes)):
            p = sizes.index(m)
            rbs, lvl = [], 0
            while True:
                try:
                    w, cap, rb = bh.tile_shape(p, lvl)
                except HB.HipBMGError:
                    break
                rbs.append(rb)
                lvl += 1
            shape[str(m)] = rbs[::-1]
        w, cap, _ = bh.tile_shape(0, 0)
        extra["batched"] = {
            "workload": "%d problems, n from {129,257,513,1025} (seed 5), lognormal D sigma=1, "
                        "FP32 V(2,1) inside FP64 refinement to rel. residual 1e-10" % args.batch,
            "problems_per_s": args.steps * args.batch / el_b,
            "ms_per_batch": 1e3 * el_b / args.steps,
            "points": npts,
            "setup_s": t_setup,
            "max_relres": max(i.relres for i in infos_b),
            "fp32_cycles_max": max(i.cycles for i in infos_b),
            "refinement_steps_max": max(i.outer_steps for i in infos_b),
            "tile_shape": {"strips_per_workgroup": w, "row_block_cap": cap,
                           "row_blocks_by_size_finest_first": shape},
        }
        log("bench: batched %.1f problems/s (%.2f ms per batch)" % (args.steps * args.batch / el_b,
                                                                   1e3 * el_b / args.steps))
        del bh, cs, bs, us

    if not args.no_adjoint:
        # gradient of 0.5 ||u(theta) - u_obs||^2 for a batch of problems:
        # theta = per-cell ln D, 5x5 box-filtered N(0,1); u_obs from a second
        # theta; forward and adjoint batched FP64 solves to 1e-10 and the
        # per-cell gradient kernel (hierarchy setup included: theta changes
        # every step of an optimisation)
        nb, m = args.adjoint_batch, 1025
        log("bench: adjoint workload (%d problems of %d^2)" % (nb, m))
        th0 = torch.stack([torch.from_numpy(inputs.theta_box5(m, m, seed=3000 + k)) for k in range(nb)]).to(dev)
        tho = torch.stack([torch.from_numpy(inputs.theta_box5(m, m, seed=4000 + k)) for k in range(nb)]).to(dev)
        ba = torch.stack([torch.from_numpy(inputs.load_uniform(m, m, seed=5000 + k)) for k in range(nb)]).to(dev)
        with torch.no_grad():
            u_obs = HB.SolveFVBatched.apply(tho, ba, TOL)
        del tho

        def grad_step():
            th = th0.clone().requires_grad_(True)
            ua = HB.SolveFVBatched.apply(th, ba, TOL)
            loss = 0.5 * ((ua - u_obs) ** 2).sum()
            loss.backward()
            return th.grad

        grad_step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            gth = grad_step()
        torch.cuda.synchronize()
        el_a = time.perf_counter() - t0
        extra["adjoint"] = {
            "workload": "%d problems of %dx%d, theta = box5(N(0,1)) per cell (seeds 3000+k), u_obs from "
                        "seeds 4000+k, loss 0.5||u-u_obs||^2, FP64 forward + adjoint to 1e-10, setup "
                        "included" % (nb, m, m),
            "gradients_per_s": args.steps * nb / el_a,
            "ms_per_batch": 1e3 * el_a / args.steps,
            "grad_abs_max": float(gth.abs().max()),
        }
        log("bench: adjoint %.1f gradients/s (%.1f ms per batch of %d)"
            % (args.steps * nb / el_a, 1e3 * el_a / args.steps, nb))
        del th0, ba, u_obs, gth

    if not args.no_3d:
        # 3D: n3^3 vertices, D constant on 8^3-cell blocks with log10 D ~ U[-2,2]
        # (seed 51), f ~ U[-1,1] (seed 53), 7-point finite volumes, V(2,1)
        # with eight-colour GS and 27-point Galerkin levels to rel. residual 1e-10
        m3 = args.n3
        log("bench: 3D workload %d^3" % m3)
        D3 = torch.from_numpy(inputs.cells3_log10_blocks(m3, m3, m3, block=8, seed=51)).to(dev)
        b3 = torch.from_numpy(inputs.load3_uniform(m3, m3, m3, seed=53)).to(dev)
        p3 = HB.fv7_from_cells(D3)
        del D3
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h3 = HB.Hierarchy3(p3)
        torch.cuda.synchronize()
        t_setup3 = time.perf_counter() - t0
        u3, i3 = h3.solve(b3, tol=TOL)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            u3, i3 = h3.solve(b3, tol=TOL)
        torch.cuda.synchronize()
        el3 = (time.perf_counter() - t0) / args.steps
        # the finest relaxation sweep (four launches: colour groups {0}, {1,2,4},
        # {3,5,6}, {7}) timed with HIP events on the solve's stream
        h3.profile(True)
        u3, i3 = h3.solve(b3, tol=TOL)
        torch.cuda.synchronize()
        pr3 = h3.profile_read()
        h3.profile(False)
        ms_r, n_r, b_r = pr3["relax_colour"]
        sweep_s = 4 * ms_r / n_r / 1e3
        # x read+written, b, W, S, B per vertex, and C unless the diagonal is
        # formed from the connections (the library counts what it moves)
        bytes_sweep = 4 * b_r
        ach3 = bytes_sweep / sweep_s / 1e9
        # each forced collapse level l* (levels 0..l* in one workgroup) against
        # the model's prediction; the largest levels are left out (seconds per solve)
        sweep3 = []
        for ls in range(min(5, i3.levels)):
            hs = HB.Hierarchy3(p3, collapse_level=ls)
            hs.solve(b3, tol=TOL)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, isw = hs.solve(b3, tol=TOL)
            torch.cuda.synchronize()
            sweep3.append({"collapse_level": ls, "measured_us_per_cycle": 1e6 * (time.perf_counter() - t0) / isw.cycles,
                           "model_us_per_cycle": i3.model_us[ls]})
            del hs
        extra["next_3d"] = {
            "workload": "%d^3 vertex 3D diffusion, D on 8^3-cell blocks log10 D~U[-2,2] (seed 51), f~U[-1,1] "
                        "(seed 53), 7-point FV, V(2,1), eight-colour GS, 27-point Galerkin levels, to rel. "
                        "residual 1e-10, FP64" % m3,
            "n": m3, "value": 1.0 / el3, "unit": "solves/s", "ms_per_solve": 1e3 * el3,
            "cycles": i3.cycles, "ms_per_cycle": 1e3 * el3 / i3.cycles, "relres": i3.relres,
            "levels": i3.levels, "setup_ms": 1e3 * t_setup3, "collapse_level": i3.collapse_level,
            "collapse_sweep": sweep3,
            "kernel_ms_per_cycle": {k: v[0] / i3.cycles for k, v in pr3.items()},
            "roofline": {"bound": "hbm", "kernel": "finest relaxation sweep (k3_gs7g<0..3>)",
                         "achieved": ach3, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": ach3 / PEAK_HBM_GBS,
                         "traffic": measured_traffic3d(), "algorithmic_bytes_per_sweep": bytes_sweep,
                         "avg_sweep_us": sweep_s * 1e6},
        }
        log("bench: 3D %.2f solves/s (%d cycles, %.3f ms/cycle), finest sweep %.1f us = %.0f GB/s algorithmic"
            % (1.0 / el3, i3.cycles, 1e3 * el3 / i3.cycles, sweep_s * 1e6, ach3))
        del h3, p3, b3, u3

    cpu = None
    if not args.no_cpu:
        from oracle import oracle as O
        nth = oracle_threads()
        log("bench: CPU oracle baseline (%d cycles on %d threads, %d on one)" % (args.cpu_cycles, nth, 2))
        planes = O.fv5(inputs.cells_log10_blocks(n, n, 16, -2.0, 2.0, seed=1))
        bh = inputs.load_uniform(n, n, seed=2)
        oh = O.Hierarchy(planes)

        def oracle_cycle_s(threads, k):
            O.set_threads(threads)
            uh = np.zeros_like(bh)
            t0 = time.perf_counter()
            for _ in range(k):
                uh = oh.vcycle(bh, uh)
            return (time.perf_counter() - t0) / k

        t_cycle = oracle_cycle_s(nth, args.cpu_cycles)
        t_cycle1 = oracle_cycle_s(1, 2)
        O.set_threads(nth)
        cpu = {"value": 1.0 / (t_cycle * cycles), "unit": "solves/s", "cores": nth, "kind": "oracle",
               "sample": "%d FP64 V(2,1)-cycles of the oracle on %d threads on the same %dx%d problem "
                         "(%.3f s/cycle), scaled by the %d cycles the solve takes; the same oracle on one "
                         "thread: 2 cycles, %.3f s/cycle" % (args.cpu_cycles, nth, n, n, t_cycle, cycles, t_cycle1),
               "single_thread_value": 1.0 / (t_cycle1 * cycles),
               "host": host_info()}
        if t_cycle * cycles <= args.cpu_solve_max_s:
            # the whole oracle solve fits the time bound: time it instead of
            # scaling a few cycles, and state the GPU solutions' error against it
            log("bench: CPU oracle, whole FP64 solve on %d threads (~%.0f s)" % (nth, t_cycle * cycles))
            t0 = time.perf_counter()
            u_or, h_or = oh.solve(bh, tol=TOL)
            t_solve = time.perf_counter() - t0
            cpu["value"] = 1.0 / t_solve
            cpu["sample"] = ("the whole FP64 solve of the oracle on %d threads on the same %dx%d problem (%d cycles, "
                             "%.1f s, relres %.2e); the same oracle on one thread: 2 cycles, %.3f s/cycle, scaled "
                             "by the cycle count" % (nth, n, n, len(h_or), t_solve, h_or[-1], t_cycle1))

            def err_vs_oracle(u):
                uh = u.cpu().numpy()
                return {"max_abs_rel": float(np.abs(uh - u_or).max() / np.abs(u_or).max()),
                        "l2_rel": float(np.linalg.norm(uh - u_or) / np.linalg.norm(u_or))}
            cpu["error_vs_oracle_solution"] = {"fp64": err_vs_oracle(u64)}
            if not args.no_mixed:
                cpu["error_vs_oracle_solution"]["mixed"] = err_vs_oracle(um)
            log("bench: error against the oracle's solution %s" % json.dumps(cpu["error_vs_oracle_solution"]))
            del u_or

    if not args.no_cpu:
        extra["cpu_oracle_workloads"] = oracle_workloads(args, n, extra, O, np, inputs)

    out = {
        "metric": "solves/s to rel. residual 1e-10, 4097^2 2D diffusion: FP64 vs FP32+refinement",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded random-block diffusivity, uniform random load)",
        "config": {"workload": "%dx%d vertex 2D diffusion, D on 16x16-cell blocks log10 D~U[-2,2], "
                               "V(2,1) to rel. residual 1e-10, Galerkin coarsening to a %dx%d direct solve, FP64"
                               % (n, n, hier.params.coarsest_n, hier.params.coarsest_n),
                   "n": n, "cycles": cycles, "levels": info.levels, "coarsest_n": hier.params.coarsest_n,
                   "collapse_level": info.collapse_level, "setup_ms": info0.setup_ms,
                   "relres": info.relres,
                   "row_blocks": {"down": list(info.rb_down)[: info.levels],
                                  "up": list(info.rb_up)[: info.levels],
                                  "pipelined_finest": info.rb_pipelined}},
        "roofline": {"bound": "hbm", "kernel": kname, "achieved": achieved, "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
                     "traffic": traffic, "algorithmic_bytes_per_launch": kbytes,
                     "avg_launch_us": kavg_s * 1e6,
                     # the relaxation's own access mix (five arrays read, one
                     # written) streamed by a probe kernel in this run's model
                     # calibration: the rate this kind of kernel can reach here
                     "access_mix_GBps": calib["hbm_GBps"],
                     "frac_of_access_mix": achieved / calib["hbm_GBps"] if calib["hbm_GBps"] > 0 else None},
        "kernels_fp64_finest": kernels,
        "model_calibration": calib,
        "redistribution_search": {"collapse_level": info.collapse_level, "stages": info.cluster_stages,
                                  "stage_workgroups": list(info.cluster_wg)[: info.cluster_stages],
                                  "stage_top_levels": list(info.cluster_hi)[: info.cluster_stages],
                                  "model_us_per_cycle": info.search_us, "states_expanded": info.search_expanded},
        "cpu_baseline": cpu,
    }
    out.update(extra)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
