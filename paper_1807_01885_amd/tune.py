"""Tune the FFT launch shape of every grid size and precision on this GPU and
write the choices to a tune cache (see cb_plan_opts.tune_cache).

    python -m paper_1807_01885_amd.tune --out paper_1807_01885_amd/tune/gfx950.txt

Plans created with tune_cache pointing at the file take the tuned shape
without timing again; TUNE_CACHE below is the one shipped for gfx950.
"""
from __future__ import annotations

import argparse
import os
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
TUNE_CACHE = os.path.join(HERE, "tune", "gfx950.txt")


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=TUNE_CACHE)
    ap.add_argument("--sizes", default="16,32,64,128,256,512,1024,2048,4096")
    a = ap.parse_args(argv)
    from . import coatbem as cb
    sizes = [int(s) for s in a.sizes.split(",")]
    # tune into a fresh file, then replace the output
    fd, tmp = tempfile.mkstemp(suffix=".txt")
    os.close(fd)
    os.unlink(tmp)
    for N in sizes:
        for prec in ("fp32", "fp64"):
            plan = cb.cb_plan_create(N, 1.0, 0.05, 20.0, 0.3, 1.0, 0.25, 0.0, prec, autotune=1, tune_cache=tmp)
            info = cb.cb_plan_get_info(plan)
            print(f"N={N:5d} {prec}: variant {info['fft_variant']} {info['tune_us']:8.2f} us", flush=True)
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    with open(tmp) as fh:
        body = fh.read()
    os.unlink(tmp)
    with open(a.out, "w") as fh:
        fh.write("# <arch> <N> <precision 0=FP64 1=FP32> <variant index> <microseconds per convolution>\n")
        fh.write(body)
    print(f"wrote {a.out}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
