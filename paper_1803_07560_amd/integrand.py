"""Drop-in integrand on the paper's line protocol (section 3, Listing 2).

Each input line holds the number of samples and the extent of the subvolume in
every dimension, ``nsamples lo1 hi1 lo2 hi2 ...``; each output line holds the
result, its absolute error and the dimension (0-based) suggested for a split::

    echo 1e7 -1 1 -1 1 | python -m paper_1803_07560_amd.integrand --integrand N-sphere --dimensions 2

Line i (0-based) is evaluated on Philox stream id ``first_id + i``.  The
evaluation runs on the GPU through ``bfi_integrand_eval``.
"""
from __future__ import annotations

import argparse
import sys

import numpy as np

from . import _binding as b
from .cli_common import add_integrand_args, integrand_of


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    add_integrand_args(ap)
    ap.add_argument("--first-id", type=int, default=1)
    args = ap.parse_args(argv)
    f = integrand_of(args)
    d = f.d
    ctx = b.bfi_context_create(0)
    try:
        for i, line in enumerate(sys.stdin):
            fields = line.split()
            if not fields:
                continue
            if len(fields) != 1 + 2 * d:
                print(f"expected 1 + 2*{d} fields, got {len(fields)}", file=sys.stderr)
                return 2
            n = int(float(fields[0]))
            ext = np.array([float(v) for v in fields[1:]]).reshape(d, 2)
            sv = b.Subvolumes([args.first_id + i], ext[:, 0], ext[:, 1], [n], [0], d)
            res, err, dim = b.bfi_integrand_eval(ctx, f, args.seed, sv)
            print(f"{res[0]:.15e} {err[0]:.15e} {int(dim[0])}", flush=True)
    finally:
        b.bfi_context_destroy(ctx)
    return 0


if __name__ == "__main__":
    sys.exit(main())
