"""Fixed workload for profiler runs (rocprofv3 kernel traces and hardware counters).

Runs the benchmark iteration (TFI ring N = 384, h = 1, 3-site clusters: 127 pair blocks
and 65 momentum blocks of 64 x 64 per iteration) for a number of steps after a warm-up,
then one plain device copy of a known size (torch's elementwise copy, 256 MiB read and
256 MiB written) whose FETCH_SIZE / WRITE_SIZE readings calibrate the byte counters.

    python paper_2106_02682_amd/profile_run.py --steps 20 [--precision fp64] [--workload c2b]

With --summarize-traffic FETCH_DIR WRITE_DIR it instead reads the counter CSVs of two
`rocprofv3 --pmc FETCH_SIZE` / `--pmc WRITE_SIZE` runs of this script, scales them by the
calibration copy's readings, and writes profiles/traffic.json (HBM bytes per launch of each
iteration kernel, tied to a digest of the eigensolver source; the benchmark reports them
only while the digest matches) and the markdown table profiles/traffic_c2b_fp64.md.
"""
import argparse
import csv
import hashlib
import json
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

COPY_BYTES = 256 << 20

# kernel name patterns of the iteration kernels (FP64 instantiations)
TRAFFIC_KERNELS = [
    ("momentum_projection", r"jacobi_kernel<vemb::cplx<double>, 64, 0, true, \d+, vemb::\(anonymous namespace\)::MomentumPolicy"),
    ("pair_projection", r"jacobi_kernel<double, 64, 0, true, \d+, vemb::\(anonymous namespace\)::PairPolicy"),
    ("projections", r"fused_projection_kernel<\d+>"),
    ("pair_update", r"pair_update_kernel"), ("pair_xstep", r"pair_xstep_kernel"),
    ("cluster_update", r"cluster_update_kernel"), ("dft_forward", r"dft_mfma_kernel<true>"),
    ("dft_inverse", r"dft_mfma_kernel<false>")]


def source_digest():
    """Digest of the eigensolver kernels' sources (jacobi.hip and its helpers)."""
    h = hashlib.sha256()
    for name in ("jacobi.hip", "jacobi_common.h"):
        with open(os.path.join(ROOT, "paper_2106_02682_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def summarize_traffic(fetch_dir, write_dir, cmd_fetch, cmd_write):
    def rows(d, counter):
        with open(os.path.join(d, "run_counter_collection.csv")) as f:
            return [r for r in csv.DictReader(f) if r["Counter_Name"] == counter]

    def calib(rs):
        copies = [r for r in rs if r["Kernel_Name"] == "__amd_rocclr_copyBuffer"]
        return float(max(copies, key=lambda r: int(r["Grid_Size"]))["Counter_Value"])

    def mean(rs, pat):
        v = [float(r["Counter_Value"]) for r in rs if re.search(pat, r["Kernel_Name"])]
        return (sum(v) / len(v) if v else None), len(v)

    F, W = rows(fetch_dir, "FETCH_SIZE"), rows(write_dir, "WRITE_SIZE")
    copy_kib = COPY_BYTES / 1024
    fF, fW = copy_kib / calib(F), copy_kib / calib(W)
    digest = source_digest()
    out = {"calibration": {"copy_bytes": COPY_BYTES, "fetch_factor": fF, "write_factor": fW,
                           "note": "FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of a plain 256 MiB device copy vs its "
                                   "true bytes"},
           "commands": {"fetch": cmd_fetch, "write": cmd_write}}
    lines = ["| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | calibrated HBM MB / launch |",
             "|---|---|---|---|---|"]
    for name, pat in TRAFFIC_KERNELS:
        (f, nf), (w, _) = mean(F, pat), mean(W, pat)
        if f is None or w is None:
            continue
        b = (f * fF + w * fW) * 1024
        out[f"{name}/fp64"] = {"bytes_per_launch": b, "fetch_kib": f, "write_kib": w, "source_digest": digest,
                               "dispatches": nf}
        lines.append(f"| {name} | {nf} | {f:.1f} | {w:.1f} | {b / 1e6:.2f} |")
    with open(os.path.join(ROOT, "profiles", "traffic.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    md = ["# HBM traffic per launch, N=384 ring, 3-site clusters (FP64)", "",
          f"Counters: `{cmd_fetch}` and `{cmd_write}` (one counter per run).", "",
          f"Calibration: a plain 256 MiB device copy (`__amd_rocclr_copyBuffer`) reads FETCH_SIZE {calib(F):.0f} KiB "
          f"and WRITE_SIZE {calib(W):.0f} KiB against {copy_kib:.0f} KiB true: factors {fF:.3f} (fetch) and "
          f"{fW:.3f} (write) are applied below.", ""] + lines + ["", f"eigensolver source digest (jacobi.hip, jacobi_common.h): {digest}",
          "Summarised by `python paper_2106_02682_amd/profile_run.py --summarize-traffic <fetch out> <write out>`."]
    with open(os.path.join(ROOT, "profiles", "traffic_c2b_fp64.md"), "w") as fh:
        fh.write("\n".join(md) + "\n")
    print("\n".join(md))


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--precision", choices=["fp64", "mixed", "fp32"], default="fp64")
    ap.add_argument("--workload", choices=["c2b", "c3a", "c3b"], default="c2b")
    ap.add_argument("--copy", type=int, default=1, help="run the calibration copy (0 skips it)")
    ap.add_argument("--summarize-traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    args = ap.parse_args()
    if args.summarize_traffic:
        cmd = ("cd /tmp && rocprofv3 --pmc {} -d <out> -o run --output-format csv -- python3 "
               "/root/repo/paper_2106_02682_amd/profile_run.py --steps 10")
        summarize_traffic(*args.summarize_traffic, cmd.format("FETCH_SIZE"), cmd.format("WRITE_SIZE"))
        return

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
