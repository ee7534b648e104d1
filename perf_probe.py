"""Workload for hardware-counter runs (rocprofv3 --pmc): a plain device copy
of known size, used to scale the counters, followed by a fixed number of FP64
V-cycles on the 4097^2 random-block problem.

    rocprofv3 --pmc FETCH_SIZE --output-format csv -d OUT_F -o run -- python3 perf_probe.py
    rocprofv3 --pmc WRITE_SIZE --output-format csv -d OUT_W -o run -- python3 perf_probe.py
    python3 perf_probe.py --summarize OUT_F OUT_W --kernel fused3

The summary step turns the two counter files into HBM bytes per launch of the
finest-level kernels, each counter scaled by what it reads for the copy
(copy bytes / counter bytes), and writes profiles/traffic.json and
profiles/traffic_fp64_4097_blocks.md.
"""
import argparse
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))


# rocprofv3 kernel names of the finest-level (5-point FP64) streaming kernels
FINEST = {
    "relax": "void hbmg::k_stream<double, 5, 0>(hbmg::StreamArgs<double>)",
    "relax_restrict": "void hbmg::k_stream<double, 5, 2>(hbmg::StreamArgs<double>)",
    "interp_relax_norm": "void hbmg::k_stream<double, 5, 5>(hbmg::StreamArgs<double>)",
    "relax2_restrict": "void hbmg::k_stream2<double, 5, false, true>(hbmg::StreamArgs<double>)",
    # the pipelined pass over a zero-excess operator (diagonal formed, not loaded)
    "fused3": "void hbmg::k_stream3<double, false, false, true, false>(hbmg::StreamArgs<double>)",
    "fused3_last": "void hbmg::k_stream3<double, true, true, true, false>(hbmg::StreamArgs<double>)",
}
# algorithmic bytes per vertex (FP64, 5-point): relaxation reads x, b, C, W, S
# and writes x; fused variants add q, the 8 weights at quarter resolution, and
# the coarse right-hand side or coarse x; the pipelined finest pass reads what
# the interpolating relaxation reads except r/C (formed from the loaded rows),
# writes the next cycle's iterate and the coarse rhs; its first stage alone
# (the last cycle of a capped run) writes the iterate instead; both form the
# diagonal of the finite-volume operator instead of reading the C plane
ALGO_B_PER_VERTEX = {"relax": 48.0, "relax_restrict": 74.0, "interp_relax_norm": 74.0,
                     "relax2_restrict": 74.0, "fused3": 60.0, "fused3_last": 58.0}


def summarize(fetch_dir, write_dir, kernel, n=4097, copy_bytes=1 << 30):
    import csv
    import hashlib
    import json
    import os

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
        for k, kn in FINEST.items():
            v = [float(r["Counter_Value"]) for r in rows if r["Kernel_Name"] == kn and r["Counter_Name"] == name]
            if v:
                per[k] = sum(v) / len(v) * 1024.0 * scale
        out[name] = {"scale": scale, "bytes_per_launch": per}
    root = os.path.dirname(os.path.abspath(__file__))
    src = os.path.join(root, "paper_1803_02481_amd", "csrc", "bmg_stream.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    npts = n * n
    lines = ["# HBM traffic of the finest-level kernels, FP64, 4097x4097 random blocks", "",
             "Commands (GPU box, `$R` = repository root):", "", "```",
             "cd /tmp && export TMPDIR=/tmp PYTHONPATH=$R",
             "rocprofv3 --pmc FETCH_SIZE --output-format csv -d $R/gpurun_out/pmc_FETCH_SIZE -o run -- "
             "python3 $R/perf_probe.py",
             "rocprofv3 --pmc WRITE_SIZE --output-format csv -d $R/gpurun_out/pmc_WRITE_SIZE -o run -- "
             "python3 $R/perf_probe.py",
             "python3 $R/perf_probe.py --summarize $R/gpurun_out/pmc_FETCH_SIZE "
             "$R/gpurun_out/pmc_WRITE_SIZE --kernel %s" % kernel, "```", "",
             "Scale factors from a 1 GiB `__amd_rocclr_copyBuffer` (bytes the copy moves / counter bytes): "
             "FETCH %.3f, WRITE %.3f." % (out["FETCH_SIZE"]["scale"], out["WRITE_SIZE"]["scale"]), "",
             "| kernel | fetch MB | write MB | HBM MB | algorithmic MB | HBM / algorithmic |",
             "|---|---|---|---|---|---|"]
    total = {}
    for k in FINEST:
        f = out["FETCH_SIZE"]["bytes_per_launch"].get(k)
        w = out["WRITE_SIZE"]["bytes_per_launch"].get(k)
        if f is None or w is None:
            continue
        algo = ALGO_B_PER_VERTEX[k] * npts
        total[k] = f + w
        lines.append("| %s | %.1f | %.1f | %.1f | %.1f | %.3f |" % (k, f / 1e6, w / 1e6, (f + w) / 1e6, algo / 1e6,
                                                                    (f + w) / algo))
    lines += ["", "Source hash of bmg_stream.hip when taken: `%s`." % sha]
    with open(os.path.join(root, "profiles", "traffic_fp64_4097_blocks.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    if kernel in total:
        with open(os.path.join(root, "profiles", "traffic.json"), "w") as fh:
            json.dump({"kernel": kernel, "source_sha": sha, "hbm_bytes_per_launch": total[kernel],
                       "all_kernels_hbm_bytes_per_launch": total}, fh, indent=1)
    print("\n".join(lines))
    return 0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--summarize", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    ap.add_argument("--kernel", default="fused3")
    ap.add_argument("--n", type=int, default=4097)
    ap.add_argument("--cycles", type=int, default=2)
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    args = ap.parse_args()
    if args.summarize:
        return summarize(args.summarize[0], args.summarize[1], args.kernel)
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
    D = torch.from_numpy(inputs.cells_log10_blocks(n, n, 16, -2.0, 2.0, seed=1)).to(dev)
    b = torch.from_numpy(inputs.load_uniform(n, n, seed=2)).to(dev)
    prec = HB.MIXED if args.precision == "mixed" else HB.FP64
    hier = HB.Hierarchy(HB.fv5_from_cells(D), max_cycles=args.cycles, precision=prec)
    _, info = hier.solve(b, tol=1e-30, check=False)
    torch.cuda.synchronize()
    print("cycles %d relres %.3e" % (info.cycles, info.relres), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
