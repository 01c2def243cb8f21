"""Writes uneven_level5_samples.json: sampled entries of the oracle's FP64
direct solution (oracle/ only) for the level-5 prolate spheroid of the
seeded uneven batch (10242 nodes, sound-soft) at two wavenumbers of its grid
k_m = 12 m / 1024, under the plane wave along +z.  At this size the oracle
takes about a minute per wavenumber, too long for a GPU test, so the test
compares the GPU result with these stored entries.

    python tests/golden/make_uneven_level5_samples.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import bie  # noqa: E402
from oracle.mesh import Surface  # noqa: E402
from workloads import uneven_bodies_workload  # noqa: E402

BODY = 2                 # the first level-5 body of the seeded batch
M_INDEX = (85, 600)      # k = 12 m / 1024
N_SAMPLES = 384


def main():
    w = uneven_bodies_workload(n_k=1024)
    body = w.bodies[BODY]
    s = Surface([body])
    assert s.n == 10242, s.n
    idx = np.sort(np.random.default_rng(2024).choice(s.n, N_SAMPLES, replace=False))
    out = {"body_index": BODY, "n": s.n, "m_index": list(M_INDEX),
           "k": [float(w.k[m - 1]) for m in M_INDEX], "sample_index": idx.tolist(),
           "x_re": [], "x_im": [], "x_norm": []}
    for m in M_INDEX:
        k = float(w.k[m - 1])
        p, dp = bie.incident_plane_wave(s, k)
        _, _, xs = bie.solve(s, k, bie.known_data(s, p, dp))
        out["x_re"].append([float(v) for v in xs[idx].real])
        out["x_im"].append([float(v) for v in xs[idx].imag])
        out["x_norm"].append(float(np.linalg.norm(xs)))
        print(f"k = {k:.6f}: |x| = {out['x_norm'][-1]:.6e}", flush=True)
    with open(os.path.join(HERE, "uneven_level5_samples.json"), "w") as f:
        json.dump(out, f, indent=0)


if __name__ == "__main__":
    main()
