"""Benchmark of the HISQ even/odd Dslash and CG on one MI355X.

Workload: 32^3 x 8 lattice, smooth links exp(0.3 i H) (fat) and three-link
path products of a second smooth field (long), antiperiodic time boundary,
m = 0.01, Gaussian sources; seeded synthetic inputs (the paper's gauge
ensembles are not available).

One step = one FP64 application of the full Dslash (D_oe then D_eo) on
device-resident packed links and fields.  ``value`` is the Dslash throughput
in algorithmic GB/s: per output site 16 link matrices (288 reals) + 16
neighbour vectors read once (12 reals, the input field read once) + the
output written (6 reals) = 300 reals = 2400 B in FP64.

Printed as one JSON line; the CG time-to-solution at true residual 1e-10 and
the CPU oracle baseline are reported in the same line.
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

HBM_PEAK_GBS = 8000.0
DSLASH_REALS_PER_SITE = 288 + 12          # links + (input vector once, output)
DSLASH_FLOP_PER_SITE = 1146


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-cg", action="store_true", help="skip the CG time-to-solution legs")
    ap.add_argument("--profile", action="store_true", help="short run for rocprofv3")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the multi-GPU "
                          "halo-exchange path is not built (--gpus must be 1)"}))
        sys.exit(2)
    import numpy as np
    import torch

    import hisq_inputs as gen
    from paper_2306_01098_amd import hisq as h

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    if not os.path.exists(h.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    h.load()

    w = gen.workload_2()
    dims, t_bc, mass = w["dims"], w["t_bc"], w["mass"]
    lat = h.lattice(dims, t_bc)
    vh = int(np.prod(dims)) // 2
    ctx = h.Context(0)
    stream = torch.cuda.current_stream()

    links64 = h.pack_links_from_host(lat, "fp64", w["fat"], w["naik"], ctx=ctx)
    src_e = h.pack_field_from_host(lat, "fp64", w["src"][0], ctx=ctx)
    tmp_o = h.empty_field(lat, "fp64")
    out_e = h.empty_field(lat, "fp64")
    torch.cuda.synchronize()

    def step():
        h.hisq_dslash(lat, "fp64", 1, links64, src_e, tmp_o, ctx=ctx)
        h.hisq_dslash(lat, "fp64", 0, links64, tmp_o, out_e, ctx=ctx)

    steps = 5 if args.profile else args.steps
    warm = 2 if args.profile else args.warmup
    for _ in range(warm):
        step()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    t0.record(stream)
    for _ in range(steps):
        step()
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_total = t0.elapsed_time(t1)
    ms_per_step = ms_total / steps
    bytes_per_dslash = vh * DSLASH_REALS_PER_SITE * 8
    per_launch_s = ms_total * 1e-3 / (2 * steps)
    gbs = bytes_per_dslash / per_launch_s / 1e9

    result = {
        "metric": "HISQ Dslash GB/s (% HBM peak) at 32^3x8; CG time-to-solution at 1e-10 residual",
        "value": round(gbs, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warm,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded smooth SU(3) links, Gaussian sources)",
        "config": {"workload": "32^3x8 HISQ D_oe+D_eo, FP64, smooth links eps=0.3, m=0.01, t_bc=-1",
                   "lattice": list(dims), "sites_per_parity": vh, "nrhs": 1},
        "hbm_fraction": round(gbs / HBM_PEAK_GBS, 4),
        "gflops": round(vh * DSLASH_FLOP_PER_SITE / per_launch_s / 1e9, 1),
        "wall_s_timed_region": round(wall, 4),
        "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "dslash_kernel<FP64,FP64,NIN=1>",
                     "algorithmic_bytes_per_launch": bytes_per_dslash},
    }

    if not args.no_cpu and not args.profile:
        from oracle import hisq as O
        lat_o = O.lattice_from(w)
        src = w["src"][0]
        O.dslash(dims, t_bc, w["fat"], w["naik"], src, 1)  # load
        n = 0
        c0 = time.perf_counter()
        while time.perf_counter() - c0 < 10.0:
            O.dslash(dims, t_bc, w["fat"], w["naik"], src, 1)
            n += 1
        dt = (time.perf_counter() - c0) / n
        result["cpu_baseline"] = {
            "value": round(bytes_per_dslash / dt / 1e9, 3), "unit": "GB/s", "cores": O.num_threads(),
            "kind": "oracle",
            "sample": f"{n} FP64 D_oe applications of the oracle at 32^3x8 (~10 s), same inputs",
        }
        del lat_o

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
