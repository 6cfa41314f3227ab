"""Write the reference spectra of the large workloads' fields (lowest |lambda|).

Calls only the CPU oracle and the seeded input generators; run from the
repository root:

    python tests/golden/make_spectra.py wilson16x32_mixed 24
    python tests/golden/make_spectra.py wilson24x48 6 1e-8

Output: tests/golden/spectrum_<workload>.json with the k eigenvalues of A of
smallest magnitude (ascending), the residual ||A x - lambda x|| of each unit
eigenvector, and the wall time. The eigenvalues come from Lanczos on A^2 (scipy
eigsh) followed by a Rayleigh-Ritz step on A (oracle.ss.lowest_magnitude_eigs),
with A the explicit sparse Hermitian Wilson matrix of Sec. 4. The eigen-window
tests choose their intervals from these values and compare the eigenvalues the
library finds with them.
"""
import json
import sys
import time
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parents[2]
sys.path.insert(0, str(ROOT))

import synth  # noqa: E402
from oracle import ss, wilson  # noqa: E402


def main(name: str, k: int, tol: float = 1e-10):
    w = synth.CONFIGS[name]
    t0 = time.time()
    A = wilson.hermitian_wilson(w.gauge(), w.dims, w.kappa)
    t_build = time.time() - t0
    print(f"{name}: matrix n = {A.shape[0]}, nnz = {A.nnz}, built in {t_build:.0f} s", flush=True)
    lam, X = ss.lowest_magnitude_eigs(A, k, tol=tol)
    res = np.linalg.norm(A @ X - X * lam[None, :], axis=0)
    out = {"workload": name, "k": k, "eigsh_tol": tol, "lam": lam.tolist(), "res": res.tolist(),
           "seconds": round(time.time() - t0, 1), "build_seconds": round(t_build, 1)}
    print("lambda:", np.round(lam, 6).tolist(), "max res", float(res.max()), flush=True)
    (Path(__file__).parent / f"spectrum_{name}.json").write_text(json.dumps(out, indent=1))


if __name__ == "__main__":
    main(sys.argv[1], int(sys.argv[2]), float(sys.argv[3]) if len(sys.argv) > 3 else 1e-10)
