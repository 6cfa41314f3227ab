"""Write the stored expected values used by the full-size GPU parity tests.

Calls only the CPU oracle and the seeded input generators; run from the
repository root:  python tests/golden/make_golden.py
Output: tests/golden/wilson8.json
  * the FP64 shifted CG of the 8^4 workload (kappa 0.125, eps 0.5, seed 1, 32 line
    nodes on [-0.1, 0.1] with beta 0.25, 4 sources): per-source iterations, per-shift
    convergence iterations, and the solution entries at 16 fixed indices per
    (source, shift);
  * the certificate of those solutions by an independent route: every (source,
    shift) system solved again by CG on its normal equations (oracle.solvers.
    normal_cg, true residual below 1e-13), the largest per-shift difference
    max_i |y_i - y'_i| / max_i |y'_i| between the two routes, and the normal-
    equation solutions at the same 16 indices;
  * the 24 eigenvalues of smallest magnitude of that matrix with their residuals,
    which the windowed eigen tests use as the reference spectrum.
"""
import json
import sys
import time
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parents[2]
sys.path.insert(0, str(ROOT))

import synth  # noqa: E402
from oracle import quadrature as quad  # noqa: E402
from oracle import solvers, ss, wilson  # noqa: E402


def main():
    w = synth.CONFIGS["wilson8_fp64"]
    t0 = time.time()
    A = wilson.hermitian_wilson(w.gauge(), w.dims, w.kappa)
    V = w.sources().reshape(w.L, -1)
    z, zeta = quad.line_nodes(w.N, w.gamma, w.rho, w.beta)
    idx = np.sort(np.random.default_rng(99).choice(w.n, 16, replace=False))
    out = {"workload": w.name, "sample_index": idx.tolist(), "sources": []}
    for l in range(w.L):
        r = solvers.shifted_cg(lambda x: A @ x, V[l], z, w.gamma, w.tol)
        tr = solvers.true_residuals(lambda x: A @ x, V[l], z, r.Y)
        Yn = solvers.normal_cg(lambda X: (A @ X.T).T, z, np.tile(V[l], (z.size, 1)), tol=1e-13)
        trn = solvers.true_residuals(lambda x: A @ x, V[l], z, Yn)
        diff = max(float(np.abs(r.Y[j] - Yn[j]).max() / np.abs(Yn[j]).max()) for j in range(z.size))
        out["sources"].append({
            "iters": int(r.iters), "status": r.status, "conv_iter": r.conv_iter.tolist(),
            "true_res_max": float(tr.max()),
            "y_sample_re": r.Y[:, idx].real.tolist(), "y_sample_im": r.Y[:, idx].imag.tolist(),
            "normal_cg_true_res_max": float(trn.max()), "normal_cg_max_rel_diff": diff,
            "yn_sample_re": Yn[:, idx].real.tolist(), "yn_sample_im": Yn[:, idx].imag.tolist()})
        print(f"source {l}: {r.iters} iterations, max true residual {tr.max():.2e}; normal-equation "
              f"route: residual {trn.max():.2e}, largest per-shift difference {diff:.2e}", flush=True)
    lam, X = ss.lowest_magnitude_eigs(A, 24)
    res = np.linalg.norm(A @ X - X * lam[None, :], axis=0)
    out["lowest_eigs"] = {"lam": lam.tolist(), "res": res.tolist(), "k": 24}
    print("lowest |lambda|:", np.round(np.sort(np.abs(lam)), 5), "max res", res.max(), flush=True)
    out["seconds"] = round(time.time() - t0, 1)
    (Path(__file__).parent / "wilson8.json").write_text(json.dumps(out))


if __name__ == "__main__":
    main()
