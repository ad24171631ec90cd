"""Standalone timing of the FP32 Wilson stencil variants (D_W, no epilogue) on one workload's
gauge field: for each variant, smpq_set_tuning then smpq_bench_dslash (two rotating buffer sets,
warm launches timed with HIP events), printing ms per launch and algorithmic GB/s.  Meant to be
run alone under a hardware-counter profiler, so that every stencil dispatch of the process is one
of the listed variants.

    python -m paper_1901_02211_amd.stencil_bench --workload noise16x32 --rhs 624 \\
        --variant 4,1,1,2 --variant 1,8,1,1

A variant is kind,rhs_per_block_or_thread,plane_band,interleave (see smpq_tuning in smpq.h).
"""
import argparse
import sys

from . import binding as smpq


def parse_variant(text):
    kind, nr, band, il = (int(v) for v in text.split(","))
    return kind, nr, band, il


def main(argv=None):
    import smpq_inputs as si

    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--workload", default="noise16x32", choices=sorted(si.WORKLOADS))
    ap.add_argument("--rhs", type=int, default=624, help="right-hand sides per launch")
    ap.add_argument("--sets", type=int, default=2, help="rotating buffer sets")
    ap.add_argument("--launches", type=int, default=10)
    ap.add_argument("--variant", action="append", type=parse_variant, required=True,
                    help="kind,nr,band,interleave")
    a = ap.parse_args(argv)
    c = smpq.smpq_create(si.WORKLOADS[a.workload]["dims"], 0)
    smpq.smpq_load_gauge(c, si.workload(a.workload))
    for kind, nr, band, il in a.variant:
        smpq.smpq_set_tuning(c, kind, nr, 1, band, 1, 1, il, 1)
        ms, by = smpq.smpq_bench_dslash(c, smpq.SMPQ_MIXED_FP32, a.rhs, a.sets, a.launches)
        print(f"kind {kind}, {nr} per block/thread, band {band}, interleave {il}: {ms:.3f} ms per launch, "
              f"{by / ms / 1e6:.0f} GB/s on {a.rhs} right-hand sides", flush=True)
    smpq.smpq_destroy(c)
    return 0


if __name__ == "__main__":
    sys.exit(main())
