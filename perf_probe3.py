"""Workload for hardware-counter runs (rocprofv3 --pmc) of the 3D path: a
plain device copy of known size, used to scale the counters, followed by a
fixed number of V-cycles on the 257^3 random-block problem.

    rocprofv3 --pmc FETCH_SIZE --output-format csv -d OUT_F -o run -- python3 perf_probe3.py
    rocprofv3 --pmc WRITE_SIZE --output-format csv -d OUT_W -o run -- python3 perf_probe3.py
    python3 perf_probe3.py --summarize OUT_F OUT_W

The summary step turns the two counter files into HBM bytes per launch of the
finest-level kernels (the launches with the largest grid of each kernel),
each counter scaled by what it reads for the copy, and writes
profiles/traffic3d.json and profiles/traffic_fp64_257cubed_blocks.md.
"""
import argparse
import os
import re
import sys

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

# finest-level kernels of the 3D path and their algorithmic bytes per vertex
# of the whole grid (FP64, 7-point, zero-excess operator: the diagonal is
# formed from the six connections, so C is not read): a colour group reads x,
# b, W, S, B and writes x at its share of the vertices (1/8 or 3/8); the
# residual reads the same and writes r; the interpolation reads x, r, C, the
# 3.25 weights per vertex and the coarse x (1/8) and writes x; the restriction
# reads r and the weights and writes the coarse rhs and the zero coarse
# iterate (1/8 each)
SWEEP_B = 48.0
KERNELS3 = {
    "gs7g<0>": ("k3_gs7g<0, true>", SWEEP_B / 8),
    "gs7g<1>": ("k3_gs7g<1, true>", SWEEP_B * 3 / 8),
    "gs7g<2>": ("k3_gs7g<2, true>", SWEEP_B * 3 / 8),
    "gs7g<3>": ("k3_gs7g<3, true>", SWEEP_B / 8),
    "resid": ("k3_resid<7, true, false, true>", 48.0),
    "resid_norm": ("k3_resid<7, false, true, true>", 40.0),
    "restrict": ("k3_restrict", 8.0 + 26.0 + 2.0),
    "interp": ("k3_interp<7>", 8.0 * (2 + 1 + 1 + 3.25 + 0.125)),
}
SWEEP = ("gs7g<0>", "gs7g<1>", "gs7g<2>", "gs7g<3>")


def source_sha():
    import hashlib
    root = os.path.dirname(os.path.abspath(__file__))
    with open(os.path.join(root, "paper_1803_02481_amd", "csrc", "bmg3d.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def summarize(fetch_dir, write_dir, n=257, copy_bytes=1 << 30):
    import csv
    import json

    def load(d):
        rows = []
        for root, _, files in os.walk(d):
            for f in files:
                if f.endswith("counter_collection.csv"):
                    rows += list(csv.DictReader(open(os.path.join(root, f))))
        return rows

    out = {}
    for name, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = load(d)
        copy = [float(r["Counter_Value"]) for r in rows if r["Kernel_Name"] == "__amd_rocclr_copyBuffer"
                and r["Counter_Name"] == name]
        scale = copy_bytes / (max(copy) * 1024.0)
        per = {}
        for k, (pat, _) in KERNELS3.items():
            sel = [r for r in rows if pat in re.sub(r"\s+", " ", r["Kernel_Name"]) and r["Counter_Name"] == name]
            if not sel:
                continue
            gmax = max(int(r["Grid_Size"]) for r in sel)
            v = [float(r["Counter_Value"]) for r in sel if int(r["Grid_Size"]) == gmax]
            per[k] = sum(v) / len(v) * 1024.0 * scale
        out[name] = {"scale": scale, "bytes_per_launch": per}
    root = os.path.dirname(os.path.abspath(__file__))
    sha = source_sha()
    npts = n ** 3
    lines = ["# HBM traffic of the 3D finest-level kernels, FP64, 257^3 random blocks", "",
             "Commands (GPU box, `$R` = repository root):", "", "```",
             "cd /tmp && export TMPDIR=/tmp PYTHONPATH=$R",
             "rocprofv3 --pmc FETCH_SIZE --output-format csv -d $R/gpurun_out/pmc3_FETCH_SIZE -o run -- "
             "python3 $R/perf_probe3.py",
             "rocprofv3 --pmc WRITE_SIZE --output-format csv -d $R/gpurun_out/pmc3_WRITE_SIZE -o run -- "
             "python3 $R/perf_probe3.py",
             "python3 $R/perf_probe3.py --summarize $R/gpurun_out/pmc3_FETCH_SIZE "
             "$R/gpurun_out/pmc3_WRITE_SIZE", "```", "",
             "Scale factors from a 1 GiB `__amd_rocclr_copyBuffer` (bytes the copy moves / counter bytes): "
             "FETCH %.3f, WRITE %.3f." % (out["FETCH_SIZE"]["scale"], out["WRITE_SIZE"]["scale"]), "",
             "| kernel | fetch MB | write MB | HBM MB | algorithmic MB | HBM / algorithmic |",
             "|---|---|---|---|---|---|"]
    total = {}
    for k, (_, bpv) in KERNELS3.items():
        f = out["FETCH_SIZE"]["bytes_per_launch"].get(k)
        w = out["WRITE_SIZE"]["bytes_per_launch"].get(k)
        if f is None or w is None:
            continue
        algo = bpv * npts
        total[k] = f + w
        lines.append("| %s | %.1f | %.1f | %.1f | %.1f | %.3f |" % (k, f / 1e6, w / 1e6, (f + w) / 1e6, algo / 1e6,
                                                                    (f + w) / algo))
    sweep = sum(total[k] for k in SWEEP) if all(k in total for k in SWEEP) else None
    if sweep is not None:
        lines += ["", "One relaxation sweep (the four colour-group launches): %.1f MB of HBM traffic against "
                      "%.1f MB algorithmic (%.3f)." % (sweep / 1e6, SWEEP_B * npts / 1e6, sweep / (SWEEP_B * npts))]
    lines += ["", "Source hash of bmg3d.hip when taken: `%s`." % sha]
    with open(os.path.join(root, "profiles", "traffic_fp64_257cubed_blocks.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    with open(os.path.join(root, "profiles", "traffic3d.json"), "w") as fh:
        json.dump({"source_sha": sha, "sweep_hbm_bytes": sweep, "hbm_bytes_per_launch": total}, fh, indent=1)
    print("\n".join(lines))
    return 0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--summarize", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    ap.add_argument("--n", type=int, default=257)
    ap.add_argument("--cycles", type=int, default=2)
    ap.add_argument("--copy-mib", type=int, default=1024)
    args = ap.parse_args()
    if args.summarize:
        return summarize(args.summarize[0], args.summarize[1], args.n)
    import torch
    from paper_1803_02481_amd import hipbmg as HB
    from paper_1803_02481_amd import inputs

    dev = "cuda:0"
    nbytes = args.copy_mib << 20
    src = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)                       # plain copy: reads and writes nbytes
    torch.cuda.synchronize()
    print("copy_bytes %d" % nbytes, flush=True)
    del src, dst
    n = args.n
    D = torch.from_numpy(inputs.cells3_log10_blocks(n, n, n, block=8, seed=51)).to(dev)
    b = torch.from_numpy(inputs.load3_uniform(n, n, n, seed=53)).to(dev)
    # eager launches (a graph replay hides its kernels from per-dispatch counters)
    hier = HB.Hierarchy3(HB.fv7_from_cells(D), max_cycles=args.cycles, use_graph=0)
    _, info = hier.solve(b, tol=1e-30, check=False)
    torch.cuda.synchronize()
    print("cycles %d relres %.3e" % (info.cycles, info.relres), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
