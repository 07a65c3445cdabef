"""Writes kf_reference_12x12.json: the coherent energy of the stationary KF
(Sec. 2.2, oracle side) on the seeded reference loop of the input generator
(workload.reference_loop), the comparison value of the benchmark's loss line
(Sec. 5: loss = (E_coh^KF - E_coh) / E_coh^KF).  Calls only the oracle and the
input generator.  Run from the repository root:  python tests/golden/make_kf_reference.py"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import geometry as geo  # noqa: E402
from oracle import kalman  # noqa: E402
from oracle import metrics as M  # noqa: E402
from paper_1408_7069_amd import workload as wl  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "kf_reference_12x12.json")


def kf_reference():
    c = wl.reference_loop()
    N, a = c["n_sub"], c["a"]
    G = geo.geometry_for(N, None)
    ij = G.node_coords()
    truth = np.array([g[ij[:, 0], ij[:, 1]] for g in c["truth"]])
    Cg = wl.vk_covariance(2 * (N + 1), c["pitch"], c["r0"], c["L0"])
    d = np.abs(ij[:, None, :] - ij[None, :, :])
    Sv = (1 - a * a) * Cg[d[..., 0], d[..., 1]]
    D = np.stack([geo.apply_slopes(G, e) for e in np.eye(G.n_nodes)], axis=1)
    r = np.full(G.n_slopes, c["sigma"] ** 2)
    _, res = kalman.closed_loop(D, truth, list(c["noise"]), Sv, r, a)
    b = c["burn_in"]
    return {"system": "12x12 SH square, a = 0.999, slope noise variance 0.04 rad^2, r0 0.15 m, "
                      "pitch 0.4 m, L0 25 m (workload.reference_loop, seed 2024)",
            "frames": int(len(res)), "burn_in": int(b),
            "residual_variance_kf": float(np.mean([M.spatial_variance(x) for x in res[b:]])),
            "e_coh_kf": M.coherent_energy(res[b:])}


if __name__ == "__main__":
    ref = kf_reference()
    with open(OUT, "w") as fh:
        json.dump(ref, fh, indent=1)
    print(json.dumps(ref))
