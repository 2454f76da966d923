"""Host-only checks of the adaptive refinement policy (``bfi_adaptive_decide``):
fed per-leaf records built from the oracle's sums, it must
  * take the leaves with the largest contribution to the variance of C until
    `refine_fraction` of the total is covered (ties by lower id),
  * split along the dimension minimising sigma_lower + sigma_upper, computed
    here by brute force from the oracle's per-sample weights,
  * double the samples instead when a split gains little and n <= n_max / 2,
    and split when doubling would exceed n_max.
No GPU: the policy is host code."""
import copy

import numpy as np
import pytest

import oracle
import workloads


def records(nx, nt, sv, seed, nu=0.7):
    lat = oracle.lattice(nx, nt, nu=nu)
    sums = oracle.sums(lat, seed, sv.ids, sv.lo, sv.hi, sv.n, sv.offset)
    spl = oracle.split_sums(lat, seed, sv.ids, sv.lo, sv.hi, sv.n, sv.offset)
    ns = len(sv)
    part = np.zeros((ns, 4 + 3 * nx))
    part[:, 0] = sums[:, 0]
    part[:, 2:] = sums[:, 1:]
    split = np.concatenate([np.zeros((ns, 1)), spl], axis=1)
    return lat, sums, part, split


def contributions(nx, d, sv, sums):
    res = oracle.finalize(nx, d, sv.lo, sv.hi, sums)
    Z, C = res["Z"], res["C"]
    V = np.prod(sv.hi - sv.lo, axis=1)
    n = sums[:, 0]
    nn = n * (n - 1)
    sw, sw2 = sums[:, 1], sums[:, 2]
    var_z = V**2 * (sw2 - sw * sw / n) / nn
    e = np.zeros(len(sv))
    for r in range(nx):
        spw, spw2, spww = sums[:, 3 + r], sums[:, 3 + nx + r], sums[:, 3 + 2 * nx + r]
        var_n = V**2 * (spw2 - spw * spw / n) / nn
        cov = V**2 * (spww - spw * sw / n) / nn
        e += var_n - 2 * C[r] * cov + C[r] ** 2 * var_z
    return np.maximum(e, 0) / Z**2


def brute_force_split(lat, seed, sv, s, count=None):
    d = lat.d
    n = int(sv.n[s]) if count is None else min(int(sv.n[s]), count)
    U = oracle.points(d, seed, int(sv.ids[s]), sv.lo[s], sv.hi[s], range(n))
    w = np.exp(-oracle.action_batch(lat, U))
    mid = 0.5 * (sv.lo[s] + sv.hi[s])
    n = len(w)
    sig = np.sqrt(max(np.mean(w * w) - np.mean(w) ** 2, 0))
    best, best_j = np.inf, 0
    for j in range(d):
        up = U[:, j] >= mid[j]
        su, qu = w[up].sum(), (w[up] ** 2).sum()
        sl, ql = w[~up].sum(), (w[~up] ** 2).sum()
        h = n / 2
        vu = max(qu / h - (su / h) ** 2, 0)
        vl = max(ql / h - (sl / h) ** 2, 0)
        sj = np.sqrt(vu) + np.sqrt(vl)
        if sj < best:
            best, best_j = sj, j
    return best_j, best / (2 * sig) if sig > 0 else 1.0


@pytest.mark.parametrize("fraction", [0.3, 0.5, 1.0])
def test_selection_and_split_dimension(bfi, fraction):
    nx, nt, seed = 3, 2, 4
    sv = workloads.random_partition(6, 2.0, 10, per_sub=1, seed=5)
    sv.n[:] = [400, 800, 1600, 400, 3200, 800, 1600, 400, 800, 6400]
    lat, sums, part, split = records(nx, nt, sv, seed)
    cfg = bfi.adaptive_config(target_rel_err=1e-6, n_min=256, n_max=1 << 20,
                              refine_fraction=fraction)
    act = bfi.bfi_adaptive_decide(bfi.lattice(nx, nt, nu=0.7), sv, part, split, cfg)
    e = contributions(nx, 6, sv, sums)
    order = sorted(range(len(sv)), key=lambda i: (-e[i], int(sv.ids[i])))
    taken, want = 0.0, set()
    for k, i in enumerate(order):
        if k > 0 and taken >= fraction * e.sum():
            break
        taken += e[i]
        want.add(i)
    assert set(np.nonzero(act >= 0)[0]) == want
    for i in want:
        j, gain = brute_force_split(lat, seed, sv, i)
        if act[i] >= 1:
            assert act[i] - 1 == j
            assert gain < 0.9
        else:
            assert act[i] == 0 and gain >= 0.9 - 1e-9


def test_split_statistics_of_first_samples(bfi):
    """With split statistics over the first m samples of each leaf (what the
    driver gathers when split_samples = m), the split dimension and gain come
    from those m samples alone, judged against their own spread (split_base);
    the ranking still uses every sample.  Without split_base the same
    statistics would be judged against the spread of all n samples."""
    nx, nt, seed, m = 3, 2, 4, 300
    sv = workloads.random_partition(6, 2.0, 10, per_sub=1, seed=5)
    sv.n[:] = [400, 800, 1600, 400, 3200, 800, 1600, 400, 800, 6400]
    lat, sums, part, _ = records(nx, nt, sv, seed)
    head = copy.deepcopy(sv)
    head.n[:] = np.minimum(sv.n, m)
    _, _, base, split = records(nx, nt, head, seed)
    cfg = bfi.adaptive_config(target_rel_err=1e-6, n_min=256, n_max=1 << 20, refine_fraction=1.0)
    act = bfi.bfi_adaptive_decide(bfi.lattice(nx, nt, nu=0.7), sv, part, split, cfg,
                                  split_base=base)
    e = contributions(nx, 6, sv, sums)
    assert set(np.nonzero(act >= 0)[0]) == set(np.nonzero(e > 0)[0])
    for i in np.nonzero(act >= 0)[0]:
        j, gain = brute_force_split(lat, seed, sv, i, count=m)
        if act[i] >= 1:
            assert act[i] - 1 == j
            assert gain < 0.9
        else:
            assert act[i] == 0 and gain >= 0.9 - 1e-9
    # split_base equal to the partials is the default
    np.testing.assert_array_equal(
        bfi.bfi_adaptive_decide(bfi.lattice(nx, nt, nu=0.7), sv, part, split, cfg,
                                split_base=part),
        bfi.bfi_adaptive_decide(bfi.lattice(nx, nt, nu=0.7), sv, part, split, cfg))


def test_split_forced_at_n_max(bfi):
    nx, nt = 2, 2
    sv = workloads.uniform_partition(4, 2.0, 2, per_sub=2048)
    lat, sums, part, split = records(nx, nt, sv, 2)
    cfg = bfi.adaptive_config(target_rel_err=1e-6, n_min=64, n_max=2048, refine_fraction=1.0)
    act = bfi.bfi_adaptive_decide(bfi.lattice(nx, nt, nu=0.7), sv, part, split, cfg)
    assert np.all(act >= 1)        # no room to double: every taken leaf splits
    cfg = bfi.adaptive_config(target_rel_err=1e-6, n_min=64, n_max=1 << 30, refine_fraction=1.0)
    act = bfi.bfi_adaptive_decide(bfi.lattice(nx, nt, nu=0.7), sv, part, split, cfg)
    assert np.all(act >= 0)


def test_decide_rejects_bad_config(bfi):
    sv = workloads.uniform_partition(4, 2.0, 1, per_sub=100)
    lat, sums, part, split = records(2, 2, sv, 1)
    for bad in (dict(n_min=1), dict(n_min=100, n_max=10), dict(refine_fraction=0.0),
                dict(target_rel_err=0.0), dict(min_ess=-1.0), dict(min_ess=float("nan")),
                dict(split_samples=1)):
        cfg = bfi.adaptive_config(**bad)
        with pytest.raises(bfi.BfiError):
            bfi.bfi_adaptive_decide(bfi.lattice(2, 2), sv, part, split, cfg)
    cfg = bfi.adaptive_config()
    cfg.holdout = 2
    with pytest.raises(bfi.BfiError):
        bfi.bfi_adaptive_decide(bfi.lattice(2, 2), sv, part, split, cfg)
