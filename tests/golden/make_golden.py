"""Write the oracle's results for the large parity cases to tests/golden/.

Calls only the FP64 oracle (oracle/) on inputs from the seeded generator
(synth/); nothing here touches the GPU library.  Usage:

    python tests/golden/make_golden.py c1 1000 1001     # n = 1000 workload
    python tests/golden/make_golden.py c2 2000          # n = 4000 workload

Each case is written to tests/golden/fram_<config>_seed<seed>.json with the
run parameters, the permutation, the objective, the accuracy against the
hidden correspondence and the per-iteration SDSN pass counts and deltas.
"""
from __future__ import annotations

import json
import pathlib
import sys
import time

import numpy as np

ROOT = pathlib.Path(__file__).resolve().parents[2]
sys.path.insert(0, str(ROOT))

import synth  # noqa: E402
from oracle import fram64 as O  # noqa: E402

# Run parameters of the parity cases: theta = 2 (dense graphs), alpha = 0.95,
# gamma_th = 1e-6, SDSN cap 1000; n = 1000 runs a fixed 100 iterations, n = 4000
# stops at delta <= 1e-6 (cap 100).
PARAMS = {
    "c1": dict(config=1, theta=2.0, alpha=0.95, iters=100, tol=0.0, gamma_th=1e-6, sdsn_max=1000),
    "c2": dict(config=2, theta=2.0, alpha=0.95, iters=100, tol=1e-6, gamma_th=1e-6, sdsn_max=1000),
}


def run(case: str, seed: int) -> pathlib.Path:
    p = PARAMS[case]
    idx = seed - 1000 * p["config"]
    pair = next(synth.config_pairs(p["config"], [idx]))
    t0 = time.time()
    N, info = O.fram(pair.A, pair.B, p["theta"], p["alpha"], p["iters"], p["tol"],
                     p["gamma_th"], p["sdsn_max"])
    sigma = O.discretize(N)
    obj = O.objective(pair.A, pair.B, sigma)
    rows = np.arange(pair.n)
    srt = np.sort(N, axis=1)
    rec = dict(
        case=case, seed=seed, n=pair.n, **p,
        perm=[int(x) for x in sigma],
        objective=obj,
        accuracy=O.accuracy(sigma, pair.perm, pair.inlier),
        outer_iters=info.outer_iters,
        converged=info.converged,
        sdsn_passes=info.sdsn_passes,
        deltas=[float(d) for d in info.deltas],
        final_gamma=float(info.gammas[-1]),
        row_argmax_is_perm=bool(len(set(np.argmax(N, axis=1))) == pair.n),
        min_row_margin=float(np.min(srt[:, -1] - srt[:, -2])),
        objective_at_truth=O.objective(pair.A, pair.B, pair.perm),
        seconds=time.time() - t0,
    )
    del rows
    out = ROOT / "tests" / "golden" / f"fram_{case}_seed{seed}.json"
    out.write_text(json.dumps(rec, indent=0))
    print(f"wrote {out} in {rec['seconds']:.0f}s: obj={obj:.6f} acc={rec['accuracy']:.4f} "
          f"iters={info.outer_iters}", flush=True)
    return out


if __name__ == "__main__":
    case = sys.argv[1]
    for s in sys.argv[2:]:
        run(case, int(s))
