"""Host-side construction of the arterial-venous coupling (Sec. 3), marshalled
to the library's C ABI (``hl_coupling_map``, ``hl_velocity_factors``).

* ``coupling_map``: the greedy distance-based mapping described in Sec. 3.
  Arterial outlets are visited in index order; each takes the closest venous
  inlet that is still free (ties: lowest inlet index), so every outlet gets at
  least one vein when there are at least as many veins.  Every vein left over
  then goes to its closest outlet.  The result is a 1:N map with the distance
  of each pair, which Eq. (1) uses as L_i.
* ``velocity_factors``: Eq. (2), the velocity scale factor v_i/v_0 of each of
  the N veins of one outlet from the pressure-drop factors dP_i/P_0, the
  distances L_i and the areas A_i (vein) and A_0 (outlet).
* ``build_pairs``: both together, giving the argument lists of ``hl_couple``.

The arithmetic of both runs in the library (host code, no device needed);
the exchange itself (forward and reverse boundary values each step) runs in
its kernels.
"""
from __future__ import annotations

import numpy as np

from . import hl_coupling_map, hl_velocity_factors


def coupling_map(outlet_centres, inlet_centres):
    """Return (outlet_of_inlet int array, distance float array), one entry per
    venous inlet; centres are (n, 3) arrays."""
    owner, dist = hl_coupling_map(outlet_centres, inlet_centres)
    return owner.astype(np.int64), dist


def velocity_factors(dp, L, A, A0):
    """Eq. (2) for the veins of one arterial outlet."""
    return hl_velocity_factors(dp, L, A, A0)


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
