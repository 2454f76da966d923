"""The allocation-free entry point bfi_eval_noalloc, through the C ABI, against
bfi_eval (same kernels and launch shape: bitwise equal records) and against the
FP64 oracle (sums within 1e-10 of their L1 scale), on two calls in a row, the
second with a smaller input, so the second call runs over what the first left
in the shared scratch array."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


def _unshift(part, nx):
    sig = part[:, 1]
    f1, f2 = np.exp(-sig), np.exp(-2 * sig)
    out = np.zeros((part.shape[0], 3 + 3 * nx))
    out[:, 0] = part[:, 0]
    out[:, 1] = part[:, 2] * f1
    out[:, 2] = part[:, 3] * f2
    out[:, 3:3 + nx] = part[:, 4:4 + nx] * f1[:, None]
    out[:, 3 + nx:3 + 3 * nx] = part[:, 4 + nx:4 + 3 * nx] * f2[:, None]
    return out


def _close_to_oracle(got, want, nx, rtol):
    assert np.array_equal(got[:, 0], want[:, 0])
    n = want[:, 0:1]
    pw2 = want[:, 3 + nx:3 + 2 * nx]
    scale = np.concatenate([want[:, 1:3], np.sqrt(n * pw2), pw2,
                            np.sqrt(pw2) * np.sqrt(want[:, 2:3])], axis=1)
    err = np.abs(got[:, 1:] - want[:, 1:])
    assert np.all(err <= rtol * scale + 1e-300), (err / (scale + 1e-300)).max()


def _cases():
    # call 1: 24 leaves of an uneven tree, counts spanning several items plus
    # ragged tails, offsets up to 2^33; call 2: fewer leaves, fewer samples
    big = workloads.random_partition(20, 4.0, 24, per_sub=1, seed=11)
    big.n[:] = workloads.log_uniform_counts(24, 1, 17, seed=5)
    big.n[:4] = [2, 3, 16383, 16385]
    big.offset[:] = np.arange(24, dtype=np.uint64) * np.uint64(2**28 + 3)
    small = workloads.random_partition(20, 4.0, 5, per_sub=1, seed=12)
    small.n[:] = [2, 100, 4097, 70000, 9]
    return big, small


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_equals_eval_two_calls(bfi, ctx, prec):
    lat = bfi.lattice(10, 2, nu=0.7)
    lat_o = oracle.lattice(10, 2, nu=0.7)
    launch = bfi.launch(samples_per_thread=16, block=64, persistent=1)
    for call, sv in enumerate(_cases()):
        print(f"noalloc: call {call} {prec} {len(sv)} subvolumes {int(sv.n.sum())} samples",
              flush=True)
        got = bfi.bfi_eval_noalloc(ctx, lat, prec, 3, sv, launch)
        ref = bfi.bfi_eval(ctx, lat, prec, 3, sv, launch)
        assert np.array_equal(got.view(np.uint64), ref.view(np.uint64)), call
        want = oracle.sums(lat_o, 3, sv.ids, sv.lo, sv.hi, sv.n, sv.offset)
        _close_to_oracle(_unshift(got, 10), want, 10, 1e-10 if prec == "fp64" else 1e-4)


def test_noalloc_split_statistics_and_grid_launch(bfi, ctx):
    """Split statistics (4x2) and one block per item, also bitwise equal to
    bfi_eval; first call larger than the second."""
    lat = bfi.lattice(4, 2)
    for call, (k, per) in enumerate(((5, 3000), (2, 700))):
        sv = workloads.uniform_partition(8, 4.0, k, per_sub=per)
        for launch in (None, bfi.launch(samples_per_thread=4, block=128, persistent=0)):
            print(f"noalloc: split call {call} launch {launch}", flush=True)
            got, gs = bfi.bfi_eval_noalloc(ctx, lat, "fp64", 1, sv, launch, split=True)
            ref, rs = bfi.bfi_eval(ctx, lat, "fp64", 1, sv, launch, split=True)
            assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))
            assert np.array_equal(gs.view(np.uint64), rs.view(np.uint64))


def test_noalloc_full_4x2_workload_and_limits(bfi, ctx):
    """The whole 4x2 workload (2^20 points, 16 subvolumes) against the oracle;
    a layout beyond the scratch array is refused with EINVAL before any launch,
    and the entry point still works after the refusal."""
    w = workloads.WORKLOADS["burgers4x2"]
    sv = workloads.uniform_partition(w.d, w.box, w.split_log2, w.budget // w.n_sub)
    lat = bfi.lattice(4, 2)
    got = bfi.bfi_eval_noalloc(ctx, lat, "fp64", w.seed, sv)
    want = oracle.sums(oracle.lattice(4, 2), w.seed, sv.ids, sv.lo, sv.hi, sv.n, sv.offset)
    _close_to_oracle(_unshift(got, 4), want, 4, 1e-10)
    # 2^22 work items of 64 samples need far more than the array holds
    huge = workloads.uniform_partition(8, 4.0, 4, per_sub=1 << 24)
    with pytest.raises(bfi.BfiError) as e:
        bfi.bfi_eval_noalloc(ctx, lat, "fp64", 1, huge, bfi.launch(samples_per_thread=1, block=64))
    assert e.value.status == -1 and "scratch" in str(e.value)
    again = bfi.bfi_eval_noalloc(ctx, lat, "fp64", w.seed, sv)
    assert np.array_equal(again.view(np.uint64), got.view(np.uint64))
