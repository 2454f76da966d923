"""Command-line adapters: integrand names and flags map to the right integrand
(host only; no GPU call)."""
import pytest

from paper_1803_07560_amd import _binding as b
from paper_1803_07560_amd import hdintegrator, integrand
from paper_1803_07560_amd.cli_common import integrand_of


def parse(argv, mod=integrand):
    import argparse
    from paper_1803_07560_amd.cli_common import add_integrand_args
    ap = argparse.ArgumentParser()
    add_integrand_args(ap)
    return ap.parse_args(argv)


def test_nsphere_by_path():
    f = integrand_of(parse(["--integrand", "integrands/N-sphere", "--dimensions", "3"]))
    assert f.kind == b.BFI_INTEGRAND_NSPHERE and f.d == 3


def test_burgers_kinds():
    z = integrand_of(parse(["--integrand", "burgers-z", "--nx", "10", "--nt", "2", "--nu", "0.5"]))
    assert z.kind == b.BFI_INTEGRAND_BURGERS_Z and z.d == 20 and z.lat.nu == 0.5
    n = integrand_of(parse(["--integrand", "burgers-n", "--distance", "5", "--precision",
                            "fp32"]))
    assert n.kind == b.BFI_INTEGRAND_BURGERS_N and n.distance == 5 and n.prec == 1


def test_bad_integrand():
    with pytest.raises(SystemExit):
        integrand_of(parse(["--integrand", "nope"]))
    with pytest.raises(SystemExit):
        integrand_of(parse(["--integrand", "N-sphere"]))


def test_modules_have_entry_points():
    assert callable(integrand.main) and callable(hdintegrator.main)
