"""Write tests/golden/spectra.json: exact low spectra of the named workloads.

The paper builds the contour from exact spectral information (Section 4); this
script computes it with the oracle's dense eigendecomposition (float64 LAPACK)
for each seeded workload and stores lambda_1..lambda_{N+8} of the unshifted H,
the canonical shift and a fingerprint of V.  Run:

    python -m oracle.make_spectra [name ...]
"""

from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

from paper_1603_09724_amd import inputs
from . import hamiltonian as ham

OUT = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "tests", "golden", "spectra.json")

WORKLOADS = {
    "well4_2d_m32_N8": lambda: inputs.small_2d(),
    "lattice8_2d_m128_N64": lambda: inputs.lattice_2d(),
}


def v_fingerprint(V: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(V, dtype=np.float64).tobytes()).hexdigest()[:16]


def spectrum_record(inst, extra: int = 8) -> dict:
    t = time.time()
    w, _ = ham.eigh_dense(inst.dim, inst.m, inst.V, 0.0, count=inst.N + extra)
    lo, hi = ham.spectral_bounds(inst.dim, inst.m, inst.V)
    return {
        "dim": inst.dim, "m": inst.m, "N": inst.N, "seed": inst.seed,
        "v_sha256_16": v_fingerprint(inst.V),
        "lambda": [float(x) for x in w],
        "lo": lo, "hi": hi, "sigma": hi + 1.0,
        "seconds": time.time() - t,
    }


def main(names):
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    for name in names or WORKLOADS:
        inst = WORKLOADS[name]()
        data[name] = spectrum_record(inst)
        print(name, "gap", data[name]["lambda"][inst.N] - data[name]["lambda"][inst.N - 1],
              "seconds", data[name]["seconds"], flush=True)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1)


if __name__ == "__main__":
    main(sys.argv[1:])
