"""The certified t-SVDM-II selection (Algorithm 2; Section 4.1: many slices
are discarded entirely) replaces the squared singular values of a slice that
gets no SVD by one stand-in, the slice's energy.  This pins the argument on
the CPU with the oracle's exact selection: whenever every stand-in lies
strictly below the tau selected from the mixed list, that tau and every rank
equal the full selection's (the skipped slices get rank 0); and the check
does fail when a stand-in reaches tau, so it is not vacuous."""
import numpy as np

import oracle as O


def _spectra(rng, r, n, quiet):
    """Squared singular values (r x n): a few loud slices with decaying
    spectra and `quiet` slices of tiny energy."""
    sq = np.empty((r, n))
    for i in range(n):
        scale = 1e-9 if i < quiet else rng.uniform(0.5, 2.0)
        sq[:, i] = np.sort(scale * rng.uniform(0.0, 1.0, r) * np.logspace(0, -6, r))[::-1]
    return sq


def _lumped(sq, skip):
    out = sq.copy()
    for i in np.flatnonzero(skip):
        e = sq[:, i].sum()
        out[:, i] = 0.0
        out[0, i] = e
    return out


def test_certified_selection_equals_full_selection():
    rng = np.random.default_rng(3)
    certified_cases = 0
    for trial in range(40):
        r, n = int(rng.integers(2, 9)), int(rng.integers(4, 30))
        sq = _spectra(rng, r, n, quiet=int(rng.integers(0, n)))
        eps = float(rng.choice([1e-3, 1e-2, 3e-2, 1e-1]))
        E = sq.sum(axis=0)
        # skip the lowest-energy slices holding half the budget
        order = np.argsort(E, kind="stable")
        cs = np.cumsum(E[order])
        skip = np.zeros(n, bool)
        skip[order[cs < 0.5 * eps * eps * E.sum()]] = True
        rho_l, info_l = O.ranks_tolerance(_lumped(sq, skip), eps, squared=True)
        if skip.any() and not np.all(E[skip] < info_l["tau"]):
            continue
        certified_cases += 1
        rho_f, info_f = O.ranks_tolerance(sq, eps, squared=True)
        assert info_l["tau"] == info_f["tau"]
        assert np.array_equal(rho_l, rho_f)
        assert np.all(rho_l[skip] == 0)
    assert certified_cases >= 20


def test_certification_can_fail():
    # one skipped slice holds a value far above the others: its stand-in
    # reaches tau, so the mixed-list selection is not trusted
    sq = np.array([[1.0, 1e-3, 2e-5], [0.5, 1e-4, 1e-6]])
    E = sq.sum(axis=0)
    skip = np.array([False, True, False])
    rho_l, info_l = O.ranks_tolerance(_lumped(sq, skip), 3e-2, squared=True)
    assert not np.all(E[skip] < info_l["tau"])
