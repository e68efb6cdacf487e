"""Writes oracle_densities.json: FP64 oracle ground states (Algorithm 1) of reduced grids of the
pancake and cigar workloads run to ||r||_inf <= 1e-10 from the seeded guesses the GPU tests use,
stored as the density |phi|^2 at 4096 seeded grid points plus its max and the max's location,
its h^3-weighted L2 norm, E and mu. Calls only oracle/ and the shared input generators.
Run: python tests/golden/make_oracle_densities.py"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import bec_inputs as bi  # noqa: E402
from oracle.energy import Model  # noqa: E402
from oracle.pcg import pcg  # noqa: E402

CASES = [("cigar_128", (32, 32, 64)), ("pancake_256", (64, 64, 16))]
TOL = 1e-10
SAMPLES = 4096


def sample_index(n, seed=2603):
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(int(np.prod(n)), size=SAMPLES, replace=False))


def main():
    out = {"_source": f"oracle.pcg.pcg (FP64 NumPy), tol ||r||_inf <= {TOL}, defaults of Algorithm 1; density "
                      f"|phi|^2 at {SAMPLES} flat C-order indices from numpy default_rng(2603)"}
    for name, n in CASES:
        w = bi.WORKLOADS[name]
        m = Model.from_workload(w, n=n)
        t = time.time()
        r = pcg(m, bi.initial_guess(w, n), tol_res=TOL)
        rho = (np.abs(r.phi) ** 2).reshape(-1)
        idx = sample_index(n)
        e = r.energies
        out[f"{name}@{n[0]}x{n[1]}x{n[2]}"] = dict(
            status=r.status, iters=r.iters, res_inf=r.res_inf, E=e.E, mu=e.mu, tol=TOL,
            rho_max=float(rho.max()), argmax=int(rho.argmax()), rho_l2=float(np.sqrt(m.grid.h3 * np.sum(rho * rho))),
            index=[int(i) for i in idx], rho=[float(v) for v in rho[idx]], seconds=time.time() - t)
        print(name, n, r.status, r.iters, r.res_inf, e.E, time.time() - t, flush=True)
    with open(os.path.join(os.path.dirname(__file__), "oracle_densities.json"), "w") as fh:
        json.dump(out, fh)


if __name__ == "__main__":
    main()
