"""Argument handling shared by the integrand and wrapper command lines."""
from __future__ import annotations

import argparse
import os

from . import _binding as b


def add_integrand_args(ap: argparse.ArgumentParser) -> None:
    ap.add_argument("--integrand", required=True,
                    help="N-sphere (any path ending in N-sphere), burgers-z (exp(-S)) or "
                         "burgers-n (u_{0,0} u_{0,r} exp(-S))")
    ap.add_argument("--dimensions", type=int, help="N-sphere: integration dimensions")
    ap.add_argument("--nx", type=int, default=10, help="lattice: space sites (M)")
    ap.add_argument("--nt", type=int, default=2, help="lattice: time slices (L)")
    ap.add_argument("--nu", type=float, default=1.0)
    ap.add_argument("--D", type=float, default=1.0)
    ap.add_argument("--a", type=float, default=1.0)
    ap.add_argument("--tau", type=float, default=1.0)
    ap.add_argument("--distance", type=int, default=0, help="burgers-n: r")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--seed", type=int, default=1)


def integrand_of(args) -> b.bfi_integrand:
    name = os.path.basename(args.integrand.rstrip("/")).lower()
    if name == "n-sphere":
        if not args.dimensions:
            raise SystemExit("--dimensions is required for the N-sphere integrand")
        return b.integrand_nsphere(args.dimensions)
    lat = b.lattice(args.nx, args.nt, nu=args.nu, D=args.D, a=args.a, tau=args.tau)
    if name == "burgers-z":
        return b.integrand_burgers(lat, args.precision)
    if name == "burgers-n":
        return b.integrand_burgers(lat, args.precision, args.distance)
    raise SystemExit(f"unknown integrand {args.integrand!r}")
