"""The paper's subdivision driver with its command-line flags (section 3,
Listing 1; criteria of sections 3 and 4), running on one GPU::

    python -m paper_1803_07560_amd.hdintegrator --integrand integrands/N-sphere \\
        --dimensions 3 --min-extent -1 --max-extent 1

prints ``result abserr``.  Every open subvolume is evaluated with --samples
and then with --sample-factor times more; it is accepted when the relative
difference is within --rel-diff (e.g. 1.025), or the absolute difference within
--abs-diff, or both results within --max-abs (a threshold <= 0 is off), and
otherwise split along the integrand's suggested dimension.
"""
from __future__ import annotations

import argparse
import sys

from . import _binding as b
from .cli_common import add_integrand_args, integrand_of


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    add_integrand_args(ap)
    ap.add_argument("--min-extent", type=float, required=True)
    ap.add_argument("--max-extent", type=float, required=True)
    ap.add_argument("--samples", type=float, default=1e6)
    ap.add_argument("--sample-factor", type=float, default=2.0)
    ap.add_argument("--rel-diff", type=float, default=1.025)
    ap.add_argument("--abs-diff", type=float, default=0.0)
    ap.add_argument("--max-abs", type=float, default=0.0)
    ap.add_argument("--split-log2", type=int, default=0)
    ap.add_argument("--max-depth", type=int, default=20)
    ap.add_argument("--max-evals", type=float, default=2.0**34)
    ap.add_argument("--stats", action="store_true", help="also print run statistics to stderr")
    args = ap.parse_args(argv)
    f = integrand_of(args)
    cfg = b.hdi_config(int(args.samples), args.sample_factor, args.rel_diff, args.abs_diff,
                       args.max_abs, args.split_log2, args.max_depth, int(args.max_evals))
    ctx = b.bfi_context_create(0)
    try:
        out = b.bfi_integrate_hdi(ctx, f, args.seed, args.min_extent, args.max_extent, cfg)
    finally:
        b.bfi_context_destroy(ctx)
    print(f"{out['result']!r} {out['abserr']!r}", flush=True)
    if args.stats:
        print({k: v for k, v in out.items() if k not in ("result", "abserr")}, file=sys.stderr)
    return 0


if __name__ == "__main__":
    sys.exit(main())
