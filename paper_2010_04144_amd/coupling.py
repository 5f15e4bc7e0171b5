"""Host-side construction of the arterial-venous coupling (Sec. 3).

* ``coupling_map``: the greedy distance-based mapping described in Sec. 3.
  Arterial outlets are visited in index order; each takes the closest venous
  inlet that is still free (ties: lowest inlet index), so every outlet gets at
  least one vein when there are at least as many veins.  Every vein left over
  then goes to its closest outlet.  The result is a 1:N map with the distance
  of each pair, which Eq. (1) uses as L_i.
* ``velocity_factors``: Eq. (2), the velocity scale factor v_i/v_0 of each of
  the N veins of one outlet from the pressure-drop factors dP_i/P_0, the
  distances L_i and the areas A_i (vein) and A_0 (outlet).  It follows from
  dP_i = k_i q_i L_i with k_i proportional to 1/A_i and q_0 = sum_i q_i.
* ``build_pairs``: both together, giving the argument lists of ``hl_couple``.

These produce the inputs of the device-side exchange; the exchange itself
(forward and reverse boundary values each step) runs in the library.
"""
from __future__ import annotations

import numpy as np


def coupling_map(outlet_centres, inlet_centres):
    """Return (outlet_of_inlet int array, distance float array), one entry per
    venous inlet."""
    a = np.asarray(outlet_centres, dtype=np.float64).reshape(-1, 3)
    v = np.asarray(inlet_centres, dtype=np.float64).reshape(-1, 3)
    na, nv = a.shape[0], v.shape[0]
    dist = np.sqrt(((a[:, None, :] - v[None, :, :]) ** 2).sum(-1))
    owner = np.full(nv, -1, dtype=np.int64)
    free = np.ones(nv, dtype=bool)
    for i in range(na):
        if not free.any():
            break
        cand = np.where(free, dist[i], np.inf)
        j = int(np.argmin(cand))          # lowest index among equal distances
        owner[j] = i
        free[j] = False
    for j in np.flatnonzero(free):
        owner[j] = int(np.argmin(dist[:, j]))
    return owner, dist[owner, np.arange(nv)]


def velocity_factors(dp, L, A, A0):
    """Eq. (2) for the veins of one arterial outlet (first vein as the
    reference of the ratios, as printed)."""
    dp = np.asarray(dp, dtype=np.float64)
    L = np.asarray(L, dtype=np.float64)
    A = np.asarray(A, dtype=np.float64)
    r = (dp * L[0] * A) / (dp[0] * L * A[0])
    return (A0 / A) * r / r.sum()


def build_pairs(dom_a, outlets, outlet_centres, outlet_areas, dom_b, inlets, inlet_centres, inlet_areas, dp):
    """Pairs (dom_a, outlet, dom_b, inlet, s_vel, dp_ratio) for ``hl_couple``.
    ``dp`` holds dP_i/P_0 per venous inlet (the paper draws it uniformly from
    [0.3, 0.7); the caller supplies the numbers)."""
    owner, L = coupling_map(outlet_centres, inlet_centres)
    dp = np.asarray(dp, dtype=np.float64)
    pairs = []
    for i in range(len(outlets)):
        js = np.flatnonzero(owner == i)
        if js.size == 0:
            continue
        s = velocity_factors(dp[js], L[js], np.asarray(inlet_areas, float)[js], float(outlet_areas[i]))
        for j, sv in zip(js, s):
            pairs.append((dom_a, int(outlets[i]), dom_b, int(inlets[j]), float(sv), float(dp[j])))
    return pairs
