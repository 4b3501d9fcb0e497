"""Fixed workload for profiler runs (rocprofv3 kernel traces and hardware counters).

Runs the benchmark iteration (TFI ring N = 384, h = 1, 3-site clusters: 127 pair blocks
and 65 momentum blocks of 64 x 64 per iteration) for a number of steps after a warm-up,
then one plain device copy of a known size (torch's elementwise copy, 256 MiB read and
256 MiB written) whose FETCH_SIZE / WRITE_SIZE readings calibrate the byte counters.

    python paper_2106_02682_amd/profile_run.py --steps 20 [--precision fp64] [--workload c2b]
"""
import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

COPY_BYTES = 256 << 20


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--precision", choices=["fp64", "mixed", "fp32"], default="fp64")
    ap.add_argument("--workload", choices=["c2b", "c3a", "c3b"], default="c2b")
    ap.add_argument("--copy", type=int, default=1, help="run the calibration copy (0 skips it)")
    args = ap.parse_args()

    import torch

    import synth
    from paper_2106_02682_amd import vemb

    torch.cuda.set_device(0)
    w = {"c2b": lambda: synth.config_c2(1.0)[1], "c3a": lambda: synth.config_c3()[0],
         "c3b": lambda: synth.config_c3()[1]}[args.workload]()
    with vemb.Problem.from_workload(w, precision=args.precision) as g:
        g.step(args.warmup)
        torch.cuda.synchronize()
        print(f"profile_run: {w.name} {args.precision}, {args.warmup} warm-up steps done", flush=True)
        g.step(args.steps)
        lb = g.dual_bound()
        torch.cuda.synchronize()
        print(f"profile_run: {args.steps} steps done, bound {lb:.12f}", flush=True)
    if args.copy:
        x = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(f"profile_run: calibration copy of {COPY_BYTES} bytes done", flush=True)


if __name__ == "__main__":
    main()
