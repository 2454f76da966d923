"""GPU: checkpoint and resume of a run over a fixed subvolume list.

Points are addressed by (seed, subvolume id, sample index), so a run resumed
from a saved state continues the same streams:
  * resumed (save, load, advance) == the same chunks run without a checkpoint,
    bit for bit;
  * the merged records equal a single evaluation of the whole range within
    the FP64 bar, and the oracle's sums of that range;
  * the FP32 form resumes the same way (bitwise against its own chunks) and
    stays within its 1e-4 bar of FP64.
"""
import numpy as np
import pytest

import oracle
import workloads
from paper_1803_07560_amd import checkpoint
from test_gpu_parity import assert_result_close, assert_sums_close, unshift

pytestmark = pytest.mark.gpu


def _case(bfi):
    nx, nt, seed = 10, 2, 17
    lat = bfi.lattice(nx, nt, nu=0.8)
    sv = workloads.uniform_partition(nx * nt, 3.0, 6, per_sub=20_000)
    more = (np.arange(len(sv), dtype=np.uint64) % 5 + 1) * np.uint64(7_001)
    return nx, nt, seed, lat, sv, more


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_resume_equals_uninterrupted_bitwise(bfi, ctx, tmp_path, prec):
    nx, nt, seed, lat, sv, more = _case(bfi)
    first = checkpoint.start(ctx, lat, prec, seed, sv)
    path = str(tmp_path / "state.json")
    checkpoint.save(first, path)
    resumed = checkpoint.advance(ctx, checkpoint.load(path), more)
    straight = checkpoint.advance(ctx, first, more)
    assert np.array_equal(resumed.partials, straight.partials)
    assert np.array_equal(resumed.subs.n, sv.n + more)
    assert np.array_equal(resumed.subs.offset, sv.offset)
    # and a second checkpoint in the middle changes nothing either
    checkpoint.save(resumed, path)
    again = checkpoint.advance(ctx, checkpoint.load(path), 4096)
    assert np.array_equal(again.partials, checkpoint.advance(ctx, straight, 4096).partials)


def test_resumed_records_match_single_pass_and_oracle(bfi, ctx):
    nx, nt, seed, lat, sv, more = _case(bfi)
    st = checkpoint.advance(ctx, checkpoint.start(ctx, lat, "fp64", seed, sv), more)
    whole = bfi.Subvolumes(sv.ids, sv.lo, sv.hi, sv.n + more, sv.offset, nx * nt)
    single = bfi.bfi_eval(ctx, lat, "fp64", seed, whole)
    assert np.array_equal(st.partials[:, 0], single[:, 0])
    assert_sums_close(unshift(st.partials, nx), unshift(single, nx), nx, 1e-12)
    pick = np.array([0, 13, 63])
    want = oracle.sums(oracle.lattice(nx, nt, nu=0.8), seed, sv.ids[pick], sv.lo[pick],
                       sv.hi[pick], whole.n[pick], 0)
    assert_sums_close(unshift(st.partials[pick], nx), want, nx, 1e-10)
    assert_result_close(checkpoint.result(st), bfi.bfi_finalize(lat, whole, single), 1e-10)


def test_fp32_form_resumes_within_bar(bfi, ctx):
    nx, nt, seed, lat, sv, more = _case(bfi)
    r64 = checkpoint.advance(ctx, checkpoint.start(ctx, lat, "fp64", seed, sv), more)
    r32 = checkpoint.advance(ctx, checkpoint.start(ctx, lat, "fp32", seed, sv), more)
    assert np.array_equal(r32.partials[:, 0], r64.partials[:, 0])
    assert_result_close(checkpoint.result(r32), checkpoint.result(r64), 1e-4)


def test_resume_far_into_the_stream(bfi, ctx):
    """A state whose samples start at index 2^40 continues from there."""
    nx, nt, seed = 4, 2, 3
    lat = bfi.lattice(nx, nt, nu=0.8)
    sv = workloads.uniform_partition(nx * nt, 2.0, 2, per_sub=5000, offset=2**40)
    st = checkpoint.advance(ctx, checkpoint.start(ctx, lat, "fp64", seed, sv), 3000)
    want = oracle.sums(oracle.lattice(nx, nt, nu=0.8), seed, sv.ids, sv.lo, sv.hi, 8000, 2**40)
    assert_sums_close(unshift(st.partials, nx), want, nx, 1e-10)
