"""GPU parity: the HIP path, called through the C ABI, against the FP64 oracle
on the same seeded inputs.

Bars:
  * Philox words and points: bit-exact (FP64 form); the FP32 form's point is the
    FP64 point to within one FP32 rounding of the map.
  * Action S: relative 1e-13 in FP64 (the kernel evaluates the residual in a
    rearranged but algebraically equal form); 1e-5 in the FP32 form.
  * Per-subvolume sums: relative 1e-10 of each sum's L1 scale (sample order and
    reduction tree differ from the oracle's sequential order).
  * Z and C(r) against the oracle: Z (through log Z) within 1e-6 relative, C(r)
    within 1e-6 of its L1 scale sum_s V_s/n_s sum |p_r w| / Z from the oracle's
    L1 sums, in FP64; 1e-4 in the FP32 form (assert_result_close_l1).  GPU-vs-GPU
    comparisons in other files measure C(r) against |C(0)|, an empirical scale.
The benchmark's workloads at full size are in test_gpu_workloads.py.
"""
import numpy as np
import pytest

import oracle
import parity_util
import workloads

pytestmark = pytest.mark.gpu

F64, F32 = "fp64", "fp32"


def unshift(part, nx):
    """bfi partial records -> oracle sums layout [n, w, w2, pw, pw2, pww]."""
    sig = part[:, 1]
    f1, f2 = np.exp(-sig), np.exp(-2 * sig)
    out = np.zeros((part.shape[0], 3 + 3 * nx))
    out[:, 0] = part[:, 0]
    out[:, 1] = part[:, 2] * f1
    out[:, 2] = part[:, 3] * f2
    out[:, 3:3 + nx] = part[:, 4:4 + nx] * f1[:, None]
    out[:, 3 + nx:3 + 3 * nx] = part[:, 4 + nx:4 + 3 * nx] * f2[:, None]
    return out


def assert_sums_close(got, want, nx, rtol):
    """Compare sums records elementwise against L1 scales: w and w^2 are
    positive; |sum p w| <= sqrt(n sum (p w)^2) and |sum p w^2| <=
    sqrt(sum (p w)^2 sum w^2) by Cauchy-Schwarz."""
    assert np.array_equal(got[:, 0], want[:, 0])
    n = want[:, 0:1]
    pw2 = want[:, 3 + nx:3 + 2 * nx]
    # product of square roots: sqrt(pw2 * w2) underflows for weights near 1e-100
    scale = np.concatenate([want[:, 1:3], np.sqrt(n * pw2), pw2,
                            np.sqrt(pw2) * np.sqrt(want[:, 2:3])], axis=1)
    err = np.abs(got[:, 1:] - want[:, 1:])
    bad = err > rtol * scale + 1e-300
    assert not bad.any(), (np.argwhere(bad)[:5], (err / (scale + 1e-300)).max())
    return float((err / (scale + 1e-300)).max())


def assert_result_close(got, want, tol):
    """Z and C(r) within tol, C(r) measured against |C(0)|.  |C(0)| is an
    empirical scale, not a bound of the L1 scale sum |p_r| w / sum w (with few
    effective samples sum u_r^2 w can exceed sum u_0^2 w); the oracle
    comparisons of this file use assert_result_close_l1 instead."""
    assert got["log_Z"] == pytest.approx(want["log_Z"], abs=tol)
    assert abs(got["Z"] - want["Z"]) <= tol * want["Z"]
    c0 = abs(want["C"][0])
    assert np.all(np.abs(got["C"] - want["C"]) <= tol * c0), (got["C"], want["C"])


def assert_result_close_l1(got, want, tol, lat_o, sv, seed):
    """Z, C(r) and C_err against the oracle's result, C(r) against its L1 scale
    from the oracle's L1 sums over the same points."""
    rec = oracle.sums_l1(lat_o, seed, sv.ids, sv.lo, sv.hi, sv.n, sv.offset)
    L = oracle.sums_len(lat_o.nx)
    scale = parity_util.c_scale(sv.lo, sv.hi, rec[:, :L], rec[:, L:])
    parity_util.assert_result_close(got, want, scale, tol)


# ---------------------------------------------------------------- points

@pytest.mark.parametrize("d", [1, 3, 4, 8, 20, 64])
def test_points_bit_exact(bfi, ctx, d):
    rng = np.random.Generator(np.random.PCG64(d))
    for sub_id, seed in [(1, 1), (1037, 1), (2**33 + 5, 2**40 + 3), (2**64 - 1, 0)]:
        lo = rng.uniform(-4, 0, size=d)
        hi = lo + rng.choice([0.5, 1.0, 4.0, 8.0], size=d)
        idx = np.array([0, 1, 2, 1023, 2**20 - 1, 2**32 + 7, 2**45 + 11], dtype=np.uint64)
        got = bfi.bfi_debug_points(ctx, d, F64, seed, sub_id, lo, hi, idx)
        want = np.stack([oracle.point(d, seed, sub_id, lo, hi, int(i)) for i in idx])
        assert np.array_equal(got.view(np.uint64), want.view(np.uint64)), (sub_id, seed)
        assert np.all(got > lo) and np.all(got < hi)


def test_fp32_points_round_the_fp64_point(bfi, ctx):
    d = 20
    lo, hi = np.full(d, -4.0), np.full(d, 4.0)
    idx = np.arange(0, 4096, dtype=np.uint64)
    p64 = bfi.bfi_debug_points(ctx, d, F64, 1, 1024, lo, hi, idx)
    p32 = bfi.bfi_debug_points(ctx, d, F32, 1, 1024, lo, hi, idx)
    assert np.all(p32 == p32.astype(np.float32))
    # (float)x rounds the word to 24 bits, then one FP32 fma: within 2 FP32 ulps of 4
    assert np.max(np.abs(p32 - p64)) <= 2 * 2.0**-21


# ---------------------------------------------------------------- action

SHAPES = [(1, 1), (1, 2), (2, 1), (2, 2), (3, 1), (3, 2), (4, 1), (4, 2), (5, 3), (8, 2),
          (10, 2), (16, 4)]


@pytest.mark.parametrize("nx,nt", SHAPES)
def test_action_matches_oracle(bfi, ctx, nx, nt):
    rng = np.random.Generator(np.random.PCG64(100 + nx * nt))
    d = nx * nt
    for params in [dict(), dict(nu=0.37, D=1.7, a=0.8, tau=0.6), dict(g=0.0, m2=0.5),
                   dict(nu=0.05, D=0.5, m2=1.25)]:
        lat_o = oracle.lattice(nx, nt, **params)
        lat_g = bfi.lattice(nx, nt, **params)
        U = rng.uniform(-4, 4, size=(300, d))
        want = oracle.action_batch(lat_o, U)
        got = bfi.bfi_debug_action(ctx, lat_g, F64, U)
        np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-13)
        got32 = bfi.bfi_debug_action(ctx, lat_g, F32, U)
        np.testing.assert_allclose(got32, want, rtol=2e-5, atol=1e-4)


def test_action_constant_field_is_zero(bfi, ctx):
    for nx, nt in [(4, 2), (10, 2), (16, 4)]:
        U = np.outer([0.0, 0.37, -3.99, 2.5], np.ones(nx * nt))
        for prec in (F64, F32):
            assert np.all(bfi.bfi_debug_action(ctx, bfi.lattice(nx, nt), prec, U) == 0.0)


# ------------------------------------------------------------- sums / eval

def oracle_and_gpu(bfi, ctx, nx, nt, sv, seed, prec=F64, launch=None, params=None, split=False):
    params = params or {}
    lat_o = oracle.lattice(nx, nt, **params)
    want = oracle.sums(lat_o, seed, sv.ids, sv.lo, sv.hi, sv.n, sv.offset)
    got = bfi.bfi_eval(ctx, bfi.lattice(nx, nt, **params), prec, seed, sv, launch, split=split)
    return lat_o, want, got


def test_config_4x2_full(bfi, ctx):
    """4x2 lattice, nu = D = 1, box [-4,4]^8, 2^20 points (seed 1) over 16
    subvolumes bisecting dims 0-3: every subvolume against the oracle."""
    w = workloads.WORKLOADS["burgers4x2"]
    sv = workloads.uniform_partition(w.d, w.box, w.split_log2, w.budget // w.n_sub)
    lat_o, want, got = oracle_and_gpu(bfi, ctx, 4, 2, sv, w.seed)
    assert_sums_close(unshift(got, 4), want, 4, 1e-10)
    res_o = oracle.finalize(4, 8, sv.lo, sv.hi, want)
    res_g = bfi.bfi_finalize(bfi.lattice(4, 2), sv, got)
    assert_result_close_l1(res_g, res_o, 1e-6, lat_o, sv, w.seed)
    np.testing.assert_allclose(res_g["C_err"], res_o["C_err"], rtol=1e-6)
    # bfi_integrate makes the same plan
    res_i = bfi.bfi_integrate(ctx, bfi.lattice(4, 2), F64, w.seed, -w.box, w.box, w.split_log2,
                              w.budget)
    assert res_i["Z"] == res_g["Z"] and np.array_equal(res_i["C"], res_g["C"])


@pytest.mark.parametrize("nx,nt", [(3, 2), (5, 3), (10, 2), (2, 1), (1, 2)])
def test_ragged_uneven_partition(bfi, ctx, nx, nt):
    """Uneven bisection tree, sample counts that are not multiples of the work
    item (2, 3, item +- 1, several items plus a tail), nonzero offsets."""
    d = nx * nt
    sv = workloads.random_partition(d, 4.0, 12, per_sub=1, seed=nx * 10 + nt)
    item = 64 * 256
    sv.n[:] = [2, 3, 255, 256, 257, item - 1, item, item + 1, 3 * item + 17, 1000, 77, 5000]
    sv.offset[:] = [0, 5, 2**20, 3, 0, 2**33, 0, 1, 7, 0, 0, 123456789]
    lat_o, want, got = oracle_and_gpu(bfi, ctx, nx, nt, sv, 7, params=dict(nu=0.6))
    assert_sums_close(unshift(got, nx), want, nx, 1e-10)


@pytest.mark.parametrize("nx,nt,obs", [(10, 2, 0), (10, 2, 1), (3, 1, 0), (16, 4, 0), (5, 3, 0)])
def test_counter_upper_word_boundaries(bfi, ctx, nx, nt, obs):
    """Work items whose Philox counters q = index * ceil(d/4) + block cross a
    multiple of 2^32 (the upper counter word changes inside the item, and for
    ceil(d/4) not a power of two inside one sample) beside items that do not:
    both kinds against the oracle, both precision forms."""
    d = nx * nt
    nb = (d + 3) // 4
    sv = workloads.random_partition(d, 3.0, 8, per_sub=1, seed=d)
    sv.n[:] = [3000, 20_000, 2, 5, 70_000, 1000, 64 * 256 + 1, 333]
    starts = []
    for k, n in zip([1, 2, 5, 7, 1, 3, 2**20, 1], sv.n):
        b = -(-(k << 32) // nb)          # first sample index with q >= k 2^32
        starts.append(b - int(n) // 2)   # the range straddles that boundary
    starts[1] = 0                        # far from any boundary
    starts[5] = 2**33 // nb              # ends short of it
    sv.offset[:] = starts
    lat_o = oracle.lattice(nx, nt, nu=0.7, observable=obs)
    want = oracle.sums(lat_o, 11, sv.ids, sv.lo, sv.hi, sv.n, sv.offset)
    lat = bfi.lattice(nx, nt, nu=0.7, observable=obs)
    got = bfi.bfi_eval(ctx, lat, F64, 11, sv, bfi.launch(8, 64, 0))
    assert_sums_close(unshift(got, nx), want, nx, 1e-10)
    got32 = bfi.bfi_eval(ctx, lat, F32, 11, sv, bfi.launch(8, 64, 1))
    assert_result_close_l1(bfi.bfi_finalize(lat, sv, got32),
                           oracle.finalize(nx, d, sv.lo, sv.hi, want), 1e-4, lat_o, sv, 11)


@pytest.mark.parametrize("nx,nt,obs", [(4, 2, 0), (10, 2, 0), (10, 2, 1), (3, 1, 0), (16, 4, 0)])
def test_mass_term_records_match_oracle(bfi, ctx, nx, nt, obs):
    """The action's mass term (m2 > 0) through the Monte Carlo kernel, whose
    sample loop is compiled with and without the term and chosen once per work
    item (d <= 32; larger lattices keep a run-time flag): records against the
    oracle in the three forms, with m2 = 0 in the same sequence of calls."""
    d = nx * nt
    sv = workloads.random_partition(d, 2.0, 6, per_sub=1, seed=d + obs)
    sv.n[:] = [2, 999, 64 * 16 + 3, 20_000, 5, 4096]
    sv.offset[:] = [0, 7, 2**20, 0, 3, 2**33]
    for m2 in (0.8, 0.0):
        params = dict(nu=0.6, m2=m2, observable=obs)
        print(f"mass term: {nx}x{nt} observable {obs} m2 {m2}", flush=True)
        lat_o = oracle.lattice(nx, nt, **params)
        want = oracle.sums(lat_o, 5, sv.ids, sv.lo, sv.hi, sv.n, sv.offset)
        lat = bfi.lattice(nx, nt, **params)
        got = bfi.bfi_eval(ctx, lat, F64, 5, sv, bfi.launch(16, 64, 1))
        assert_sums_close(unshift(got, nx), want, nx, 1e-10)
        # the shifted FP64 form (nothing underflows on this machine: its records
        # moved back to sigma = 0 are the plain sums)
        got64s = bfi.bfi_eval(ctx, lat, "fp64s", 5, sv, bfi.launch(16, 64, 1))
        assert_sums_close(unshift(got64s, nx), want, nx, 1e-10)
        got32 = bfi.bfi_eval(ctx, lat, F32, 5, sv, bfi.launch(16, 64, 1))
        assert_result_close_l1(bfi.bfi_finalize(lat, sv, got32),
                               oracle.finalize(nx, d, sv.lo, sv.hi, want), 1e-4, lat_o, sv, 5)


@pytest.mark.parametrize("launch", [
    dict(samples_per_thread=1, block=64, persistent=0),
    dict(samples_per_thread=7, block=128, persistent=0),
    dict(samples_per_thread=64, block=256, persistent=0),
    dict(samples_per_thread=64, block=256, persistent=1),
    dict(samples_per_thread=16, block=64, persistent=1),
    dict(samples_per_thread=256, block=128, persistent=1),
    dict(samples_per_thread=3, block=512, persistent=0),
    dict(samples_per_thread=64, block=512, persistent=1),
    dict(samples_per_thread=5, block=1024, persistent=0),
    dict(samples_per_thread=32, block=1024, persistent=1),
])
def test_launch_shapes_agree(bfi, ctx, launch):
    nx, nt = 10, 2
    sv = workloads.uniform_partition(20, 4.0, 5, per_sub=40_000)
    sv.n[3] = 17
    lat_o, want, got = oracle_and_gpu(bfi, ctx, nx, nt, sv, 1, launch=bfi.launch(**launch))
    assert_sums_close(unshift(got, nx), want, nx, 1e-10)


@pytest.mark.parametrize("block", [512, 1024])
def test_large_blocks_every_form(bfi, ctx, block):
    """512- and 1024-thread blocks (the 1024-thread kernels hold 128 registers
    and spill): the FP64 forms within 1e-10 of the oracle's sums, the FP32 form
    within its stated 1e-4, persistent and grid launches bit-identical."""
    nx, nt = 10, 2
    sv = workloads.random_partition(20, 4.0, 6, per_sub=50_000, seed=block)
    sv.n[1] = 2
    sv.n[4] = 3 * block * 8 + 5
    lat_o = oracle.lattice(nx, nt)
    want = oracle.sums(lat_o, 9, sv.ids, sv.lo, sv.hi, sv.n, sv.offset)
    lat = bfi.lattice(nx, nt)
    for prec in (F64, "fp64s"):
        got = bfi.bfi_eval(ctx, lat, prec, 9, sv, bfi.launch(8, block, 1))
        assert_sums_close(unshift(got, nx), want, nx, 1e-10)
        grid = bfi.bfi_eval(ctx, lat, prec, 9, sv, bfi.launch(8, block, 0))
        assert np.array_equal(grid, got)
    got32 = bfi.bfi_eval(ctx, lat, F32, 9, sv, bfi.launch(8, block, 1))
    assert_result_close_l1(bfi.bfi_finalize(lat, sv, got32),
                           oracle.finalize(nx, 20, sv.lo, sv.hi, want), 1e-4, lat_o, sv, 9)
    assert np.array_equal(bfi.bfi_eval(ctx, lat, F32, 9, sv, bfi.launch(8, block, 0)), got32)


def test_block_sizes_outside_the_compiled_set_rejected(bfi, ctx):
    sv = workloads.uniform_partition(8, 4.0, 2, per_sub=1000)
    for block in (32, 192, 384, 2048):
        with pytest.raises(bfi.BfiError):
            bfi.bfi_eval(ctx, bfi.lattice(4, 2), F64, 1, sv, bfi.launch(16, block, 1))


def test_persistent_equals_grid_bitwise(bfi, ctx):
    sv = workloads.random_partition(20, 4.0, 40, per_sub=30_000, seed=3)
    sv.n[::3] = 12_345
    a = bfi.bfi_eval(ctx, bfi.lattice(10, 2), F64, 5, sv, bfi.launch(32, 256, 0))
    b = bfi.bfi_eval(ctx, bfi.lattice(10, 2), F64, 5, sv, bfi.launch(32, 256, 1))
    c = bfi.bfi_eval(ctx, bfi.lattice(10, 2), F64, 5, sv, bfi.launch(32, 256, 1))
    assert np.array_equal(a, b) and np.array_equal(b, c)
    a32 = bfi.bfi_eval(ctx, bfi.lattice(10, 2), F32, 5, sv, bfi.launch(32, 256, 0))
    b32 = bfi.bfi_eval(ctx, bfi.lattice(10, 2), F32, 5, sv, bfi.launch(32, 256, 1))
    assert np.array_equal(a32, b32)


@pytest.mark.parametrize("nx,nt,box", [(4, 2, 4.0), (10, 2, 4.0), (10, 2, 1.0), (16, 4, 3.0),
                                        (8, 2, 4.0)])
def test_fp32_shifted_form_error(bfi, ctx, nx, nt, box):
    """FP32 action and exp, FP64 sums: Z and C(r) within 1e-4 of the FP64 oracle
    on the same points (stated bound)."""
    d = nx * nt
    sv = workloads.uniform_partition(d, box, 4, per_sub=20_000)
    lat_o, want, got = oracle_and_gpu(bfi, ctx, nx, nt, sv, 1, prec=F32)
    res_o = oracle.finalize(nx, d, sv.lo, sv.hi, want)
    res_g = bfi.bfi_finalize(bfi.lattice(nx, nt), sv, got)
    assert_result_close_l1(res_g, res_o, 1e-4, lat_o, sv, 1)
    assert np.all(np.isfinite(got))


def test_split_statistics(bfi, ctx):
    nx, nt = 10, 2
    sv = workloads.random_partition(20, 4.0, 6, per_sub=25_000, seed=11)
    sv.n[2] = 999
    for prec in (F64, F32):
        part, spl = bfi.bfi_eval(ctx, bfi.lattice(nx, nt), prec, 3, sv, None, split=True)
        want = oracle.split_sums(oracle.lattice(nx, nt), 3, sv.ids, sv.lo, sv.hi, sv.n, sv.offset)
        sig = spl[:, 0:1]
        assert np.array_equal(sig[:, 0], part[:, 1])
        got = np.concatenate([spl[:, 1:21] * np.exp(-sig), spl[:, 21:41] * np.exp(-2 * sig)], 1)
        tol = 1e-10 if prec == F64 else 1e-4
        tot = unshift(part, nx)
        scale = np.concatenate([np.repeat(tot[:, 1:2], 20, 1), np.repeat(tot[:, 2:3], 20, 1)], 1)
        assert np.all(np.abs(got - want) <= tol * scale)


def test_graph_replays_match_eager(bfi, ctx):
    nx, nt = 10, 2
    sv = workloads.uniform_partition(20, 4.0, 6, per_sub=20_000)
    lat = bfi.lattice(nx, nt)
    eager = bfi.bfi_eval(ctx, lat, F64, 9, sv, bfi.launch(64, 256, 1))
    plan = bfi.bfi_plan_create(ctx, lat, F64, sv, bfi.launch(64, 256, 1, use_graph=1))
    try:
        for rep in range(4):
            bfi.bfi_plan_run(plan, 9)
            got = bfi.bfi_plan_partials(plan, len(sv), nx)
            assert np.array_equal(got, eager), rep
            # eager work between replays
            other = bfi.bfi_eval(ctx, bfi.lattice(4, 2), F64, rep, workloads.uniform_partition(
                8, 4.0, 2, per_sub=1000))
            assert np.all(np.isfinite(other))
        bfi.bfi_plan_run(plan, 10)   # new seed: graph recaptured
        got10 = bfi.bfi_plan_partials(plan, len(sv), nx)
        assert np.array_equal(got10, bfi.bfi_eval(ctx, lat, F64, 10, sv, bfi.launch(64, 256, 1)))
    finally:
        bfi.bfi_plan_destroy(plan)


def test_graph_replays_per_destination(bfi, ctx):
    """A graph plan writing to alternating device buffers (one captured replay per
    buffer), then to six buffers in turn (more than the four replays kept):
    every replay's records equal the eager evaluation, with eager work and host
    reads between replays."""
    torch = pytest.importorskip("torch")
    nx, nt = 10, 2
    sv = workloads.uniform_partition(20, 4.0, 6, per_sub=20_000)
    lat = bfi.lattice(nx, nt)
    eager = bfi.bfi_eval(ctx, lat, F32, 4, sv, bfi.launch(64, 256, 1))
    bufs = [torch.full((len(sv), bfi.partial_len(nx)), -1.0, dtype=torch.float64,
                       device="cuda:0") for _ in range(6)]
    stream = torch.cuda.Stream()
    plan = bfi.bfi_plan_create(ctx, lat, F32, sv, bfi.launch(64, 256, 1, use_graph=1))
    try:
        for rep, b in enumerate([0, 1, 0, 1, 0, 1, 2, 3, 4, 5, 0, 1, 2]):
            bufs[b].fill_(-1.0)
            torch.cuda.synchronize()
            bfi.bfi_plan_run(plan, 4, bufs[b], stream)
            stream.synchronize()
            assert np.array_equal(bufs[b].cpu().numpy(), eager), (rep, b)
            other = bfi.bfi_eval(ctx, bfi.lattice(4, 2), F64, rep, workloads.uniform_partition(
                8, 4.0, 2, per_sub=1000))
            assert np.all(np.isfinite(other))
    finally:
        bfi.bfi_plan_destroy(plan)


def test_plan_writes_torch_buffer_on_torch_stream(bfi, ctx):
    torch = pytest.importorskip("torch")
    nx, nt = 4, 2
    sv = workloads.uniform_partition(8, 4.0, 4, per_sub=10_000)
    lat = bfi.lattice(nx, nt)
    eager = bfi.bfi_eval(ctx, lat, F64, 1, sv)
    buf = torch.zeros((len(sv), bfi.partial_len(nx)), dtype=torch.float64, device="cuda:0")
    stream = torch.cuda.Stream()
    plan = bfi.bfi_plan_create(ctx, lat, F64, sv)
    try:
        bfi.bfi_plan_run(plan, 1, buf, stream)
        stream.synchronize()
        assert np.array_equal(buf.cpu().numpy(), eager)
    finally:
        bfi.bfi_plan_destroy(plan)


# ------------------------------------------------------------------ edges

def test_invalid_arguments(bfi, ctx):
    sv = workloads.uniform_partition(8, 4.0, 1, per_sub=100)
    with pytest.raises(bfi.BfiError) as e:
        bfi.bfi_eval(ctx, bfi.lattice(7, 7), F64, 1, workloads.uniform_partition(49, 1.0, 0, 10))
    assert e.value.name == "BFI_EUNSUPPORTED"
    for bad in (dict(D=0.0), dict(nu=float("nan")), dict(a=-1.0), dict(m2=-1.0)):
        with pytest.raises(bfi.BfiError) as e:
            bfi.bfi_eval(ctx, bfi.lattice(4, 2, **bad), F64, 1, sv)
        assert e.value.name == "BFI_EINVAL"
    bad = sv.subset([0, 1])
    bad.n[0] = 1
    with pytest.raises(bfi.BfiError):
        bfi.bfi_eval(ctx, bfi.lattice(4, 2), F64, 1, bad)
    bad = sv.subset([0, 1])
    bad.hi[1, 3] = bad.lo[1, 3]
    with pytest.raises(bfi.BfiError):
        bfi.bfi_eval(ctx, bfi.lattice(4, 2), F64, 1, bad)
    with pytest.raises(bfi.BfiError):
        bfi.bfi_eval(ctx, bfi.lattice(4, 2), F64, 1, sv, bfi.launch(64, 96, 0))
    # the library stays usable after errors
    assert np.all(np.isfinite(bfi.bfi_eval(ctx, bfi.lattice(4, 2), F64, 1, sv)))
    # sample indices whose Philox counter (index * ceil(d/4) + j) would wrap
    wrap = workloads.uniform_partition(8, 4.0, 0, per_sub=100)
    wrap.offset[:] = 2**63 - 99            # last index 2^63: counter 2^64 would wrap
    with pytest.raises(bfi.BfiError) as e:
        bfi.bfi_eval(ctx, bfi.lattice(4, 2), F64, 1, wrap)
    assert e.value.name == "BFI_EINVAL"
    wrap.offset[:] = 2**63 - 100           # last index 2^63 - 1: counter 2^64 - 1, allowed
    assert np.all(np.isfinite(bfi.bfi_eval(ctx, bfi.lattice(4, 2), F64, 1, wrap)))


def test_empty_list_is_a_no_op(bfi, ctx):
    empty = workloads.uniform_partition(8, 4.0, 1, per_sub=10).subset([])
    out = bfi.bfi_eval(ctx, bfi.lattice(4, 2), F64, 1, empty)
    assert out.shape == (0, 16)


def test_minimal_subvolume_two_samples(bfi, ctx):
    sv = workloads.uniform_partition(3, 2.0, 0, per_sub=2)
    lat_o, want, got = oracle_and_gpu(bfi, ctx, 3, 1, sv, 1)
    assert_sums_close(unshift(got, 3), want, 3, 1e-12)
