"""Writes oracle_solves.json: FP64 oracle ground states (Algorithm 1) of reduced grids of the
pancake and cigar workloads, from the same seeded initial guesses the GPU tests use. Calls only
oracle/ and the shared input generators. Run: python tests/golden/make_oracle_solves.py"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import bec_inputs as bi  # noqa: E402
from oracle.energy import Model  # noqa: E402
from oracle.pcg import pcg  # noqa: E402

CASES = [("pancake_256", (64, 64, 16)), ("cigar_128", (32, 32, 64))]


def main():
    out = {"_source": "oracle.pcg.pcg (FP64 NumPy), tol ||r||_inf <= 1e-8, defaults of Algorithm 1"}
    for name, n in CASES:
        w = bi.WORKLOADS[name]
        m = Model.from_workload(w, n=n)
        t = time.time()
        r = pcg(m, bi.initial_guess(w, n))
        e = r.energies
        out[f"{name}@{n[0]}x{n[1]}x{n[2]}"] = dict(status=r.status, iters=r.iters, res_inf=r.res_inf, E=e.E, mu=e.mu,
                                                  Ekin=e.Ekin, Epot=e.Epot, Eint=e.Eint, Edip=e.Edip, Erot=e.Erot,
                                                  virial=e.virial, seconds=time.time() - t)
        print(name, n, out[f"{name}@{n[0]}x{n[1]}x{n[2]}"], flush=True)
    with open(os.path.join(os.path.dirname(__file__), "oracle_solves.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
