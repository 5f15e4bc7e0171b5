"""Host-side coupling construction (Sec. 3): the greedy mapping, checked
against its definition by brute force, and Eq. (2), checked against the
oracle's independent implementation and against mass conservation."""
import itertools

import numpy as np

from paper_2010_04144_amd import coupling


def test_mapping_properties_and_bruteforce():
    rng = np.random.default_rng(3)
    for na, nv in [(1, 1), (1, 5), (3, 3), (4, 13), (5, 26), (6, 2)]:
        a = rng.uniform(0, 100, (na, 3))
        v = rng.uniform(0, 100, (nv, 3))
        owner, L = coupling.coupling_map(a, v)
        assert owner.shape == (nv,) and np.all((owner >= 0) & (owner < na))
        if nv >= na:
            assert set(owner.tolist()) == set(range(na))      # every artery gets a vein
        d = np.sqrt(((a[:, None] - v[None]) ** 2).sum(-1))
        # first phase: arteries in index order take the nearest free vein
        free = set(range(nv))
        first = {}
        for i in range(na):
            if not free:
                break
            j = min(free, key=lambda jj: (d[i, jj], jj))
            first[j] = i
            free.discard(j)
        for j, i in first.items():
            assert owner[j] == i
        for j in free:                                          # second phase: nearest artery
            assert owner[j] == int(np.argmin(d[:, j]))
        assert np.allclose(L, d[owner, np.arange(nv)])


def test_mapping_exhaustive_tiny():
    """On every assignment of 2 arteries x 3 veins on a line, the map equals
    the definition evaluated by enumeration of the greedy choices."""
    pts = [0.0, 1.0, 2.5, 4.0, 7.0]
    for perm in itertools.permutations(pts, 5):
        a = np.array([[perm[0], 0, 0], [perm[1], 0, 0]])
        v = np.array([[perm[2], 0, 0], [perm[3], 0, 0], [perm[4], 0, 0]])
        owner, _ = coupling.coupling_map(a, v)
        d = np.abs(a[:, 0][:, None] - v[:, 0][None])
        j0 = int(np.argmin(d[0]))
        rest = [j for j in range(3) if j != j0]
        j1 = rest[int(np.argmin(d[1, rest]))]
        exp = {j0: 0, j1: 1}
        for j in range(3):
            if j not in exp:
                exp[j] = int(np.argmin(d[:, j]))
        assert owner.tolist() == [exp[j] for j in range(3)]


def test_velocity_factors_match_oracle_and_conserve_mass(oracle_mod):
    rng = np.random.default_rng(5)
    for nv in (1, 2, 3, 13):
        dp = rng.uniform(0.3, 0.7, nv)
        L = rng.uniform(5, 50, nv)
        A = rng.uniform(10, 200, nv)
        A0 = rng.uniform(50, 500)
        v = coupling.velocity_factors(dp, L, A, A0)
        np.testing.assert_allclose(v, oracle_mod.velocity_factors(dp, L, A, A0), rtol=1e-14)
        assert abs((A * v).sum() - A0) / A0 < 1e-14


def test_build_pairs_covers_every_vein():
    rng = np.random.default_rng(8)
    a = rng.uniform(0, 50, (4, 3))
    v = rng.uniform(0, 50, (52, 3))
    pairs = coupling.build_pairs(0, [1, 2, 3, 4], a, [30, 30, 30, 30], 1, list(range(52)), v,
                                 rng.uniform(5, 15, 52), rng.uniform(0.3, 0.7, 52))
    assert sorted(p[3] for p in pairs) == list(range(52))
    assert {p[1] for p in pairs} == {1, 2, 3, 4}
    for p in pairs:
        assert 0.3 <= p[5] < 0.7 and p[4] > 0
