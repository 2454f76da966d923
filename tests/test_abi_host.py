"""The C ABI library loads, exports every entry point ``include/bfi.h``
declares, and its host-only logic (shape table, validation, finalize) agrees
with the oracle.  No GPU: nothing here launches a kernel."""
import math
import os
import re
import subprocess

import numpy as np
import pytest

import oracle
import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bfi.h")


def declared_symbols():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+char\s*\*|bfi_status)\s*(bfi_\w+)\s*\(", txt,
                                 re.M)))


def test_header_declares_entry_points():
    names = declared_symbols()
    for n in ("bfi_eval", "bfi_finalize", "bfi_integrate", "bfi_integrate_adaptive",
              "bfi_plan_run", "bfi_server_submit", "bfi_debug_points", "bfi_debug_action",
              "bfi_autotune"):
        assert n in names


def test_library_exports_every_declared_symbol(bfi):
    out = subprocess.run(["nm", "-D", "--defined-only", bfi.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s+(bfi_\w+)", out))
    missing = [n for n in declared_symbols() if n not in exported]
    assert not missing, missing
    # the binding binds exactly the declared entry points
    assert sorted(bfi.EXPORTED) == declared_symbols()


def test_library_has_gfx950_code_objects(bfi):
    out = subprocess.run(["/opt/rocm/bin/roc-obj-ls", bfi.LIB_PATH], capture_output=True,
                         text=True)
    if out.returncode != 0:
        pytest.skip("roc-obj-ls unavailable")
    assert "gfx950" in out.stdout


def test_supported_shapes(bfi):
    shapes = bfi.bfi_supported_shapes()
    for s in [(4, 2), (8, 2), (10, 2), (16, 4), (1, 1), (3, 1)]:
        assert s in shapes
        assert bfi.bfi_shape_supported(*s)
    assert not bfi.bfi_shape_supported(7, 7)


def _oracle_case(nx, nt, B=2.0, k=3, per=3000, seed=3):
    lat = oracle.lattice(nx, nt, nu=0.8)
    sv = workloads.uniform_partition(nx * nt, B, k, per_sub=per)
    sums = oracle.sums(lat, seed, sv.ids, sv.lo, sv.hi, sv.n, sv.offset)
    return lat, sv, sums


def _as_partials(sums, nx, sigma):
    """Oracle sums -> bfi partial records with shift sigma per subvolume:
    first-order sums times exp(sigma), second-order times exp(2 sigma)."""
    ns = sums.shape[0]
    sig = np.broadcast_to(np.asarray(sigma, dtype=np.float64), (ns,))
    p = np.zeros((ns, 4 + 3 * nx))
    f1, f2 = np.exp(sig), np.exp(2 * sig)
    p[:, 0] = sums[:, 0]
    p[:, 1] = sig
    p[:, 2] = sums[:, 1] * f1
    p[:, 3] = sums[:, 2] * f2
    p[:, 4:4 + nx] = sums[:, 3:3 + nx] * f1[:, None]
    p[:, 4 + nx:4 + 3 * nx] = sums[:, 3 + nx:3 + 3 * nx] * f2[:, None]
    return p


@pytest.mark.parametrize("shifted", [False, True])
def test_finalize_matches_oracle(bfi, shifted):
    nx, nt = 4, 2
    lat, sv, sums = _oracle_case(nx, nt)
    want = oracle.finalize(nx, nx * nt, sv.lo, sv.hi, sums)
    sigma = np.linspace(-30, 40, len(sv)) if shifted else 0.0
    got = bfi.bfi_finalize(bfi.lattice(nx, nt, nu=0.8), sv, _as_partials(sums, nx, sigma))
    assert got["log_Z"] == pytest.approx(want["log_Z"], rel=1e-13, abs=1e-13)
    assert got["Z"] == pytest.approx(want["Z"], rel=1e-12)
    assert got["Z_err"] == pytest.approx(want["Z_err"], rel=1e-9)
    assert got["ess"] == pytest.approx(want["ess"], rel=1e-12)
    assert got["n_evals"] == want["n_evals"]
    np.testing.assert_allclose(got["C"], want["C"], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(got["C_err"], want["C_err"], rtol=1e-8)


def test_finalize_large_shift_keeps_log_z(bfi):
    """Shifts far beyond the double range still give a finite log Z and C."""
    nx, nt = 3, 1
    lat, sv, sums = _oracle_case(nx, nt, k=2)
    want = oracle.finalize(nx, nx * nt, sv.lo, sv.hi, sums)
    p = _as_partials(sums, nx, 0.0)
    p[:, 1] = -800.0            # claim the weights were exp(-800) times larger
    got = bfi.bfi_finalize(bfi.lattice(nx, nt), sv, p)
    assert got["log_Z"] == pytest.approx(want["log_Z"] + 800.0, rel=1e-13)
    np.testing.assert_allclose(got["C"], want["C"], rtol=1e-12)


def test_finalize_rejects_short_records(bfi):
    lat, sv, sums = _oracle_case(2, 1, k=1)
    p = _as_partials(sums, 2, 0.0)
    p[0, 0] = 1.0
    with pytest.raises(bfi.BfiError) as e:
        bfi.bfi_finalize(bfi.lattice(2, 1), sv, p)
    assert e.value.name == "BFI_EINVAL"


def _unshift(p, nx):
    """bfi partial records -> oracle sums layout (scaled back by the shift)."""
    sig = p[:, 1]
    f1, f2 = np.exp(-sig), np.exp(-2 * sig)
    s = np.zeros((p.shape[0], 3 + 3 * nx))
    s[:, 0] = p[:, 0]
    s[:, 1] = p[:, 2] * f1
    s[:, 2] = p[:, 3] * f2
    s[:, 3:3 + nx] = p[:, 4:4 + nx] * f1[:, None]
    s[:, 3 + nx:] = p[:, 4 + nx:] * f2[:, None]
    return s


def test_partials_merge_is_the_sum_over_both_ranges(bfi):
    """Records of [0, n) and [n, n + m), each with its own shift, merge into the
    oracle's record of [0, n + m) (disjoint sample ranges add)."""
    nx, nt, seed = 3, 2, 5
    lat = oracle.lattice(nx, nt, nu=0.8)
    sv = workloads.uniform_partition(nx * nt, 2.0, 3, per_sub=1500)
    a = oracle.sums(lat, seed, sv.ids, sv.lo, sv.hi, 1500, 0)
    b = oracle.sums(lat, seed, sv.ids, sv.lo, sv.hi, 2500, 1500)
    want = oracle.sums(lat, seed, sv.ids, sv.lo, sv.hi, 4000, 0)
    sig_a = np.linspace(-20, 30, len(sv))
    sig_b = np.linspace(25, -15, len(sv))
    got = bfi.bfi_partials_merge(nx, _as_partials(a, nx, sig_a), _as_partials(b, nx, sig_b))
    assert np.array_equal(got[:, 1], np.minimum(sig_a, sig_b))
    s = _unshift(got, nx)
    assert np.array_equal(s[:, 0], want[:, 0])
    np.testing.assert_allclose(s[:, 1:], want[:, 1:], rtol=1e-12, atol=0)


def test_partials_merge_empty_records(bfi):
    nx = 2
    lat, sv, sums = _oracle_case(nx, 1, k=1)
    full = _as_partials(sums, nx, 3.0)
    empty = np.zeros_like(full)
    empty[:, 1] = np.nan          # ignored when n = 0
    assert np.array_equal(bfi.bfi_partials_merge(nx, empty, full), full)
    assert np.array_equal(bfi.bfi_partials_merge(nx, full, empty), full)


def test_partials_merge_rejects_bad_records(bfi):
    nx = 2
    lat, sv, sums = _oracle_case(nx, 1, k=1)
    good = _as_partials(sums, nx, 0.0)
    bads = []
    frac = good.copy()
    frac[1, 0] = 10.5
    bads.append(frac)
    neg = good.copy()
    neg[0, 0] = -2.0
    bads.append(neg)
    nan_shift = good.copy()
    nan_shift[0, 1] = np.nan
    bads.append(nan_shift)
    big = good.copy()
    big[:, 0] = 2.0**53
    bads.append(big)
    for bad in bads:
        with pytest.raises(bfi.BfiError) as e:
            bfi.bfi_partials_merge(nx, good, bad)
        assert e.value.name == "BFI_EINVAL"
    acc = good.copy()
    rc = bfi.load().bfi_partials_merge(nx, acc.shape[0], bfi._binding._dp(acc),
                                       bfi._binding._dp(frac))
    assert rc == -1 and np.array_equal(acc, good)   # unchanged on error
    with pytest.raises(bfi.BfiError):
        bfi.bfi_partials_merge(0, good[:, :4], good[:, :4])


def test_checkpoint_json_round_trip_is_exact(bfi):
    """A run state survives save/load bit for bit, and its estimate is the
    oracle's for the records it holds."""
    from paper_1803_07560_amd import checkpoint
    nx, nt = 4, 2
    lat_o, sv, sums = _oracle_case(nx, nt)
    lat = bfi.lattice(nx, nt, nu=0.8, observable="averaged")
    lat.D = 0.1 + 2.0**-40
    part = _as_partials(sums, nx, np.linspace(-700.0, 3.0, len(sv)))
    subs = bfi.Subvolumes(sv.ids + np.uint64(2**63), sv.lo / 3.0, sv.hi / 7.0, sv.n,
                          sv.offset + np.uint64(2**40 + 1), nx * nt)
    st = checkpoint.RunState(lat, "fp32", 2**64 - 1, subs, part)
    back = checkpoint.from_json(checkpoint.to_json(st))
    for f in checkpoint._LATTICE_FIELDS:
        assert getattr(back.lat, f) == getattr(lat, f)
    assert back.prec == "fp32" and back.seed == 2**64 - 1
    for f in ("ids", "lo", "hi", "n", "offset"):
        assert np.array_equal(getattr(back.subs, f), getattr(subs, f))
    assert np.array_equal(back.partials, part)
    doc = checkpoint.to_json(st)
    with pytest.raises(ValueError):
        checkpoint.from_json(doc.replace('"count": 8', '"count": 9'))
    with pytest.raises(ValueError):
        checkpoint.from_json(doc.replace(checkpoint.FORMAT, "other"))


def test_checkpoint_result_matches_oracle(bfi, tmp_path):
    from paper_1803_07560_amd import checkpoint
    nx, nt = 4, 2
    lat_o, sv, sums = _oracle_case(nx, nt)
    lat = bfi.lattice(nx, nt, nu=0.8)
    st = checkpoint.RunState(lat, "fp64", 3, bfi.Subvolumes.of(sv, nx * nt),
                             _as_partials(sums, nx, 0.0))
    path = str(tmp_path / "run.json")
    checkpoint.save(st, path)
    got = checkpoint.result(checkpoint.load(path))
    want = oracle.finalize(nx, nx * nt, sv.lo, sv.hi, sums)
    assert got["log_Z"] == pytest.approx(want["log_Z"], rel=1e-13)
    np.testing.assert_allclose(got["C"], want["C"], rtol=1e-12, atol=1e-14)


def test_finalize_counts_two_evaluations_per_pair(bfi):
    nx, nt = 4, 2
    lat_o, sv, sums = _oracle_case(nx, nt)
    p = _as_partials(sums, nx, 0.0)
    single = bfi.bfi_finalize(bfi.lattice(nx, nt, nu=0.8), sv, p)
    pairs = bfi.bfi_finalize(bfi.lattice(nx, nt, nu=0.8, antithetic=True), sv, p)
    assert pairs["n_evals"] == 2 * single["n_evals"]
    assert pairs["Z"] == single["Z"] and np.array_equal(pairs["C"], single["C"])
    bad = bfi.lattice(nx, nt, nu=0.8)
    bad.antithetic = 3
    with pytest.raises(bfi.BfiError) as e:
        bfi.bfi_finalize(bad, sv, p)
    assert e.value.name == "BFI_EINVAL"


@pytest.mark.parametrize("k", [13, 15])
def test_finalize_of_many_records_matches_oracle(bfi, k):
    """Lists above one finalize chunk (8192 records) are summed in parallel
    chunks: the result equals the oracle's finalize of the same records, and
    shifted records give the same result as their rescaled plain copy."""
    nx, d = 2, 4
    sv = workloads.uniform_partition(d, 2.0, k, per_sub=10)
    rng = np.random.default_rng(k)
    m = len(sv)
    rec = np.zeros((m, 4 + 3 * nx))
    rec[:, 0] = rng.integers(2, 1000, m)
    rec[:, 2] = rng.uniform(0.5, 2.0, m) * rec[:, 0]
    rec[:, 3] = rec[:, 2] ** 2 / rec[:, 0] * rng.uniform(1.0, 3.0, m)
    rec[:, 4:6] = rng.normal(size=(m, nx)) * rec[:, 2:3]
    rec[:, 6:8] = rec[:, 4:6] ** 2 + rec[:, 3:4]
    rec[:, 8:10] = rng.normal(size=(m, nx)) * rec[:, 3:4]
    got = bfi.bfi_finalize(bfi.lattice(nx, 2), sv, rec)
    want = oracle.finalize(nx, d, sv.lo, sv.hi, np.concatenate([rec[:, :1], rec[:, 2:]], 1))
    assert got["Z"] == pytest.approx(want["Z"], rel=1e-13)
    np.testing.assert_allclose(got["C"], want["C"], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(got["C_err"], want["C_err"], rtol=1e-10)
    assert got["n_evals"] == want["n_evals"]
    shifted = rec.copy()
    shifted[:, 1] = rng.uniform(-3, 3, m)
    f1 = np.exp(shifted[:, 1])
    shifted[:, 2] *= f1
    shifted[:, 4:6] *= f1[:, None]
    shifted[:, 3] *= f1 ** 2
    shifted[:, 6:10] *= (f1 ** 2)[:, None]
    again = bfi.bfi_finalize(bfi.lattice(nx, 2), sv, shifted)
    assert again["log_Z"] == pytest.approx(got["log_Z"], abs=1e-12)
    np.testing.assert_allclose(again["C"], got["C"], rtol=1e-10, atol=1e-13)


def test_sph_finalize_matches_oracle(bfi):
    """bfi_sph_finalize weights each shell by its volume: on the oracle's own
    records it gives the oracle's finalize with shell volumes (host only)."""
    lat_o = oracle.lattice(3, 1)
    edges = np.linspace(0.0, 2.0 * math.sqrt(3.0), 7)
    ids = np.arange(1, 7, dtype=np.uint64)
    s = oracle.sph_sums(lat_o, 4, 2.0, ids, edges[:-1], edges[1:], 3000)
    ref = oracle.sph_finalize(3, 3, edges[:-1], edges[1:], s)
    part = np.zeros((6, 4 + 9))
    part[:, 0] = s[:, 0]
    part[:, 2:] = s[:, 1:]
    got = bfi.bfi_sph_finalize(bfi.lattice(3, 1), bfi.Shells(ids, edges[:-1], edges[1:], 3000),
                               part)
    assert got["Z"] == pytest.approx(ref["Z"], rel=1e-13)
    np.testing.assert_allclose(got["C"], ref["C"], rtol=1e-12)
    np.testing.assert_allclose(got["C_err"], ref["C_err"], rtol=1e-10)
