"""Workload for hardware-counter runs (rocprofv3 --pmc): a plain device copy
of known size, used to scale the counters, followed by a fixed number of FP64
V-cycles on the 4097^2 random-block problem.

    rocprofv3 --pmc FETCH_SIZE -- python3 -m paper_1803_02481_amd.perf_probe
"""
import argparse
import sys


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=4097)
    ap.add_argument("--cycles", type=int, default=2)
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    args = ap.parse_args()
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
